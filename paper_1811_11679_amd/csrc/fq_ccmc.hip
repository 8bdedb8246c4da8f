// Coupled cluster Monte Carlo (paper Sec. 2.2, eq. ccmc) on the FCIQMC path.
//
// The list holds excitor amplitudes N_i on determinants D_i = a_i D_0 up to
// the truncation level, and t_HF = N_0 on D_0. Psi_CC = N_0 exp(T / N_0) D_0,
// T = sum_i N_i a_i, expands into terms N_0^(1-s) prod N_e a_{e_1}...a_{e_s} D_0.
// The terms of zero and one excitor are the list entries themselves: they
// spawn and die in the FCIQMC kernels (whose spawns stop at the truncation
// level). The composite terms (s >= 2) are sampled here:
//
//  * k_ccmc_scan: exclusive prefix of |N_i| over the current list in its
//    order (hash, then key), the reference's entry counted as zero, by
//    decoupled look-back; it records N_0 and N_ex = sum |N_i|;
//  * k_ccmc_clusters: n_c = ceil(N_ex 2^-b) selections, one per thread. A
//    selection draws a size s in [2, s_max] (p(s) = 2^-(s-1), the largest size
//    taking the remainder 2^-(s_max-2), s_max = truncation + 2), then s
//    excitors with probability |N_i| / N_ex each (a 64-bit uniform integer r
//    maps to the entry whose prefix range holds floor(r N_ex / 2^64)). The
//    excitors are applied to D_0 one after another as second-quantised
//    moves (k-th lowest hole to k-th lowest particle, each move signed by the
//    occupied spin-orbitals between its ends, times the sign that makes
//    a_e D_0 = +D_e); the product vanishes when two excitors share a hole or
//    a particle (a repeated excitor always does). The term's weight per
//    selection is sgn N_0 (N_ex / |N_0|)^s / (p(s) s! n_c); it makes one
//    spawning attempt from the collapsed determinant D onto a D_j within the
//    truncation level and, when D is within it, adds its death step
//    -dtau (K_DD - S) w (stochastically rounded) as a spawn onto D. Records
//    join the spawned list and are annihilated with it.
//  * k_ccmc_singles / k_ccmc_pairs: the projected energy's t~_j of a double
//    holds (1 / N_0) sgn N_a N_b for every pair of singles with
//    a_a a_b D_0 = sgn D_j; the singles of the new list are queued and the
//    pair sum taken exactly (fixed-point limbs at 2^-64) into the iteration's
//    estimator record.
//
// Random numbers: Philox under the key (k0, k1 ^ 2^31), counter (tag, draw,
// t, selection index): the size and excitor draws use their own tag; the
// spawning attempt of a selection uses the blocks an attempt 0 of a parent
// with hash equal to the selection index would use.
#include "fq_kernels.h"
#include "fq_scan.h"

namespace fq {

constexpr int CC_T = 256, CC_I = 8, CC_TILE = CC_T * CC_I;
// prefix entries a cluster block stages in LDS (32 KB): lists of up to 4095
// entries are searched there, longer ones in global memory
constexpr int CC_LDS_CUM = 4096;

// ---------------------------------------------------------------------------
// prefix of |N_i| over the current list (reference masked), N_0, N_ex
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(CC_T) void k_ccmc_scan(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    const long long n = c->n_main;
    const long long ntiles = (n + CC_TILE - 1) / CC_TILE;
    const uint32_t epoch = epoch_of(c->t, 14);
    const DevSys &sy = w.sys[w.rep[0].sys];
    __shared__ long long s_v[CC_TILE];
    __shared__ long long s_red[8];
    __shared__ long long s_tile, s_base;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[TK_CCMC], 1u);
        __syncthreads();
        const long long tile = s_tile;
        if (tile >= ntiles) break;
        const long long t0 = tile * CC_TILE;
        // striped loads (coalesced): |N_i|, the reference's entry as zero
        for (int k = 0; k < CC_I; ++k) {
            const int l = k * CC_T + threadIdx.x;
            const long long i = t0 + l;
            long long a = 0;
            if (i < n) {
                const int32_t p = w.cur.pop[i];
                bool is_ref = true;
#pragma unroll
                for (int q = 0; q < W; ++q) is_ref = is_ref && w.cur.key[(size_t)q * w.main_cap + i] == sy.ref[q];
                if (is_ref)
                    c->ccmc_n0 = p;
                else
                    a = p < 0 ? -(long long)p : (long long)p;
            }
            s_v[l] = a;
        }
        __syncthreads();
        // blocked scan: thread t owns entries CC_I t .. CC_I t + CC_I - 1
        long long loc = 0;
        for (int k = 0; k < CC_I; ++k) loc += s_v[threadIdx.x * CC_I + k];
        long long tot;
        const long long ex = block_excl_scan<long long>(loc, tot, s_red);
        if (threadIdx.x < 64) {
            const long long lb = lookback(w.st_ccmc, tile, epoch, tot);
            if (threadIdx.x == 0) s_base = lb;
        }
        __syncthreads();
        {
            long long run = s_base + ex;
            for (int k = 0; k < CC_I; ++k) {
                const int l = threadIdx.x * CC_I + k;
                const long long v = s_v[l];
                s_v[l] = run;
                run += v;
            }
        }
        __syncthreads();
        for (int k = 0; k < CC_I; ++k) {
            const int l = k * CC_T + threadIdx.x;
            if (t0 + l < n) w.ccmc_cum[t0 + l] = s_v[l];
        }
        if (tile == ntiles - 1 && threadIdx.x == 0) {
            w.ccmc_cum[n] = s_base + tot;
            c->ccmc_nex = s_base + tot;
        }
        __syncthreads();
    }
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) w.ccmc_cum[0] = 0;
}

// ---------------------------------------------------------------------------
// one excitor applied to D: its moves, the k-th lowest hole to the k-th
// lowest particle, each signed by the occupied spin-orbitals strictly between
// its ends in the determinant it acts on; returns the product of the signs.
// The caller has checked that every hole is occupied and every particle empty.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ int lowest_bit(const uint64_t (&m)[W])
{
#pragma unroll
    for (int i = 0; i < W; ++i)
        if (m[i]) return 64 * i + __ffsll((unsigned long long)m[i]) - 1;
    return -1;
}

template <int W>
__device__ int apply_moves(uint64_t (&D)[W], const uint64_t (&holes)[W], const uint64_t (&parts)[W])
{
    uint64_t hm[W], pm[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        hm[i] = holes[i];
        pm[i] = parts[i];
    }
    int sign = 1;
    for (int k = 0; k < 8; ++k) {
        const int h = lowest_bit<W>(hm);
        if (h < 0) break;
        const int p = lowest_bit<W>(pm);
        if (parity_between<W>(D, h, p) < 0.0) sign = -sign;
        flipbit<W>(D, h);
        flipbit<W>(D, p);
        flipbit<W>(hm, h);
        flipbit<W>(pm, p);
    }
    return sign;
}

// ---------------------------------------------------------------------------
// composite clusters: one selection per thread, records appended to the
// spawned list (one atomic per wave on the spawn count)
// ---------------------------------------------------------------------------
template <int KIND, int W>
__global__ __launch_bounds__(CC_T) void k_ccmc_clusters(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    const RepParams &rp = w.rep[0];
    const DevSys &sy = w.sys[rp.sys];
    const long long n0 = c->ccmc_n0, nex = c->ccmc_nex;
    if (n0 == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&c->err, ERR_NOREF);
        return;
    }
    const int trunc = w.ccmc_trunc;
    const int smax = trunc + 2 < sy.nel ? trunc + 2 : sy.nel;
    const int bits = rp.bits;
    const long long nc = bits ? (nex + (1ll << bits) - 1) >> bits : nex;
    if (smax < 2 || nc == 0) return;
    const long long n = c->n_main;
    const uint32_t t = c->t;
    const uint32_t k0 = rp.k0, k1 = rp.k1 ^ 0x80000000u;
    const double an0 = (double)(n0 < 0 ? -n0 : n0);
    const double S = w.shift[0];
    uint64_t ref[W];
#pragma unroll
    for (int q = 0; q < W; ++q) ref[q] = sy.ref[q];
    const int lane = lane_id();
    const long long stride = (long long)gridDim.x * CC_T;
    // the prefix, staged in LDS when it fits (every selection searches it)
    __shared__ long long s_cum[CC_LDS_CUM];
    const bool staged = n + 1 <= CC_LDS_CUM;
    if (staged)
        for (long long i = threadIdx.x; i <= n; i += CC_T) s_cum[i] = w.ccmc_cum[i];
    __syncthreads();
    const long long *cum = staged ? s_cum : w.ccmc_cum;
    for (long long base = (long long)blockIdx.x * CC_T; base < nc; base += stride) {
        const long long sel = base + threadIdx.x;
        // up to two records: the spawn (0) and the term's death step (1)
        bool has[2] = {false, false};
        uint64_t rkey[2][W];
        int32_t ramp[2] = {0, 0};
        if (sel < nc) {
            U4 rr = draw(TAG_CLUSTER, 0, t, (uint64_t)sel, k0, k1);
            const double u = u53(rr.x, rr.y);
            int sz = 2;
            while (sz < smax && u >= 1.0 - ldexp(1.0, -(sz - 1))) ++sz;
            const double ps = sz < smax ? ldexp(1.0, -(sz - 1)) : ldexp(1.0, -(smax - 2));
            uint64_t D[W], hall[W], pall[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                D[q] = ref[q];
                hall[q] = 0;
                pall[q] = 0;
            }
            int sgn = 1;
            bool alive = true;
            for (int j = 0; j < sz && alive; ++j) {
                rr = draw(TAG_CLUSTER, 1u + (uint32_t)j, t, (uint64_t)sel, k0, k1);
                const uint64_t r64 = ((uint64_t)rr.x << 32) | (uint64_t)rr.y;
                const long long target = (long long)__umul64hi(r64, (uint64_t)nex);
                long long lo = 0, hi = n;  // last entry whose prefix is <= target
                while (hi - lo > 1) {
                    const long long mid = (lo + hi) >> 1;
                    if (cum[mid] <= target) lo = mid; else hi = mid;
                }
                uint64_t e[W], he[W], pe[W];
                bool clash = false;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    e[q] = w.cur.key[(size_t)q * w.main_cap + lo];
                    he[q] = ref[q] & ~e[q];
                    pe[q] = e[q] & ~ref[q];
                    clash = clash || (he[q] & hall[q]) != 0 || (pe[q] & pall[q]) != 0;
                }
                if (clash) {
                    alive = false;
                    break;
                }
                // a_e = sigma_e (moves of e), sigma_e fixed by a_e D_0 = +D_e
                uint64_t R0[W];
#pragma unroll
                for (int q = 0; q < W; ++q) R0[q] = ref[q];
                const int sigma = apply_moves<W>(R0, he, pe);
                const int m = apply_moves<W>(D, he, pe);
                sgn *= sigma * m;
                if (w.cur.pop[lo] < 0) sgn = -sgn;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    hall[q] |= he[q];
                    pall[q] |= pe[q];
                }
            }
            int lev = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) lev += __popcll(hall[q]);
            if (alive && lev <= trunc + 2) {
                if ((sz % 2 == 0) && n0 < 0) sgn = -sgn;  // sign of N_0^(1-s)
                const double x = (double)nex / an0;
                double f = x;
                for (int j = 1; j < sz; ++j) f = f * x;
                double fact = 1.0;
                for (int j = 2; j <= sz; ++j) fact *= (double)j;
                const double mag = (an0 * f) / ((ps * fact) * (double)nc);
                // one spawning attempt from D
                const U4 r0 = draw(TAG_SELECT, 0, t, (uint64_t)sel, k0, k1);
                double pgen = 0.0, hv = 0.0;
                uint64_t child[W];
#pragma unroll
                for (int q = 0; q < W; ++q) child[q] = 0;
                bool ok;
                if constexpr (KIND == K_HUBBARD)
                    ok = gen_hubbard<W>(sy, D, r0.x, child, pgen, hv);
                else if constexpr (KIND == K_UEG)
                    ok = gen_ueg<W>(sy.u, D, r0.x, r0.y, child, pgen, hv);
                else
                    ok = gen_heatbath<W>(sy, rp.p_single, D, r0, 0u, t, (uint64_t)sel, k0, k1, child, pgen, hv);
                if (ok && hv != 0.0) {
                    int d = 0;
#pragma unroll
                    for (int q = 0; q < W; ++q) d += __popcll(child[q] ^ ref[q]);
                    if ((d >> 1) <= trunc) {
                        const double mm = ((rp.tau * fabs(hv)) / pgen) * mag;
                        double uu;
                        if constexpr (KIND == K_MOLECULAR) {
                            const U4 rs = draw(TAG_SPAWN_ROUND, 0, t, (uint64_t)sel, k0, k1);
                            uu = u53(rs.x, rs.y);
                        } else {
                            uu = u53(r0.z, r0.w);
                        }
                        long long kk = 0;
                        if (!(mm < 0x1p31)) {
                            atomicOr(&c->err, ERR_OVERFLOW);
                        } else {
                            if (bits != 0 && mm < (double)rp.cu)
                                kk = (uu * (double)rp.cu < mm) ? rp.cu : 0;
                            else
                                kk = sround(mm, uu);
                            if (kk > 2147483647ll) {
                                atomicOr(&c->err, ERR_OVERFLOW);
                                kk = 0;
                            }
                        }
                        if (kk != 0) {
                            const int sh = hv > 0.0 ? 1 : -1;
                            ramp[0] = (int32_t)(-(long long)(sh * sgn) * kk);
                            has[0] = true;
#pragma unroll
                            for (int q = 0; q < W; ++q) rkey[0][q] = child[q];
                        }
                    }
                }
                // the term's death step, as a spawn onto D
                if (lev <= trunc) {
                    const double md = (rp.tau * ((diag_element<KIND, W>(sy, D) - sy.H00) - S)) * mag;
                    const U4 rd = draw(TAG_DEATH, 0, t, (uint64_t)sel, k0, k1);
                    const double ud = u53(rd.x, rd.y);
                    if (!(fabs(md) < 0x1p31)) {
                        atomicOr(&c->err, ERR_OVERFLOW);
                    } else {
                        const long long k = sround(fabs(md), ud);
                        if (k > 2147483647ll) atomicOr(&c->err, ERR_OVERFLOW);
                        if (k != 0 && k <= 2147483647ll) {
                            ramp[1] = (int32_t)((md >= 0.0 ? -sgn : sgn) * k);
                            has[1] = true;
#pragma unroll
                            for (int q = 0; q < W; ++q) rkey[1][q] = D[q];
                        }
                    }
                }
            }
        }
        // append: one atomic per wave on the spawn count
        const uint64_t b0 = __ballot(has[0]), b1 = __ballot(has[1]);
        const uint32_t cnt = (uint32_t)(__popcll(b0) + __popcll(b1));
        unsigned long long wbase = 0;
        if (lane == 0 && cnt) wbase = atomicAdd(&c->n_spawn, (unsigned long long)cnt);
        wbase = __shfl(wbase, 0, 64);
        if (cnt && wbase + cnt > (unsigned long long)w.spawn_cap) {
            if (lane == 0) atomicOr(&c->err, ERR_SPAWN_CAP);
            continue;
        }
        if (lane == 0 && cnt) atomicAdd((unsigned long long *)&w.acc[0].ccmc_rec, (unsigned long long)cnt);
        const uint32_t r0i = (uint32_t)__popcll(b0 & lanemask_lt());
        const uint32_t r1i = (uint32_t)__popcll(b0) + (uint32_t)__popcll(b1 & lanemask_lt());
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            if (!has[x]) continue;
            const long long o = (long long)wbase + (x == 0 ? r0i : r1i);
            w.sp.skey[o] = make_skey(hash64<W>(rkey[x]) & w.hmask, 0u, w.rb);
            uint64_t *rec = w.sp.rec + (size_t)o * (W + 1);
#pragma unroll
            for (int q = 0; q < W; ++q) rec[q] = rkey[x][q];
            rec[W] = (uint64_t)(uint32_t)ramp[x] | (1ull << 32);
        }
    }
}

// ---------------------------------------------------------------------------
// projected energy: singles of a list queued, then the exact pair sum
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(256) void k_ccmc_singles(Work w, int setup)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    const MainList L = setup ? w.cur : w.nxt;
    const long long n = setup ? c->n_main : c->n_main_new;
    const DevSys &sy = w.sys[w.rep[0].sys];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        uint64_t k[W];
        int d = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            k[q] = L.key[(size_t)q * w.main_cap + i];
            d += __popcll(k[q] ^ sy.ref[q]);
        }
        const int32_t p = L.pop[i];
        if (d != 2 || p == 0) continue;
        const uint32_t slot = atomicAdd(&c->n_single, 1u);
        if (slot >= (uint32_t)w.single_cap) continue;  // cannot happen: single_cap counts every single
#pragma unroll
        for (int q = 0; q < W; ++q) w.single_key[(size_t)q * w.single_cap + slot] = k[q];
        w.single_pop[slot] = p;
    }
}

template <int KIND, int W>
__global__ __launch_bounds__(256) void k_ccmc_pairs(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    const DevSys &sy = w.sys[w.rep[0].sys];
    const long long n1 = c->n_single < (uint32_t)w.single_cap ? c->n_single : (uint32_t)w.single_cap;
    const long long np = n1 * (n1 - 1) / 2;
    long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    uint64_t ref[W];
#pragma unroll
    for (int q = 0; q < W; ++q) ref[q] = sy.ref[q];
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < np; x += (long long)gridDim.x * blockDim.x) {
        // pair index -> (i, j), i < j: row i holds n1 - 1 - i pairs
        long long i = (long long)((2.0 * n1 - 1.0 - sqrt((2.0 * n1 - 1.0) * (2.0 * n1 - 1.0) - 8.0 * x)) * 0.5);
        if (i < 0) i = 0;
        while (i > 0 && i * (2 * n1 - i - 1) / 2 > x) --i;
        while ((i + 1) * (2 * n1 - i - 2) / 2 <= x) ++i;
        const long long j = x - i * (2 * n1 - i - 1) / 2 + i + 1;
        uint64_t D[W], ha[W], pa[W], hb[W], pb[W];
        bool clash = false;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint64_t ea = w.single_key[(size_t)q * w.single_cap + i];
            const uint64_t eb = w.single_key[(size_t)q * w.single_cap + j];
            ha[q] = ref[q] & ~ea;
            pa[q] = ea & ~ref[q];
            hb[q] = ref[q] & ~eb;
            pb[q] = eb & ~ref[q];
            clash = clash || (ha[q] & hb[q]) != 0 || (pa[q] & pb[q]) != 0;
            D[q] = ref[q];
        }
        if (clash) continue;
        uint64_t R0[W];
#pragma unroll
        for (int q = 0; q < W; ++q) R0[q] = ref[q];
        int sg = apply_moves<W>(R0, ha, pa) * apply_moves<W>(D, ha, pa);
#pragma unroll
        for (int q = 0; q < W; ++q) R0[q] = ref[q];
        sg *= apply_moves<W>(R0, hb, pb) * apply_moves<W>(D, hb, pb);
        const double h = hij<KIND, W>(sy, ref, D);
        // H_0,ab (N_a N_b): symmetric in the pair, whose order in the queue is arbitrary
        const double term = h * ((double)w.single_pop[i] * (double)w.single_pop[j]);
        add_limbs4(a0, a1, a2, a3, sg > 0 ? term : -term);
    }
    a0 = wave_sum<long long>(a0);
    a1 = wave_sum<long long>(a1);
    a2 = wave_sum<long long>(a2);
    a3 = wave_sum<long long>(a3);
    if (lane_id() == 0 && (a0 | a1 | a2 | a3)) {
        atomicAdd((unsigned long long *)&w.acc[0].pair[0], (unsigned long long)a0);
        atomicAdd((unsigned long long *)&w.acc[0].pair[1], (unsigned long long)a1);
        atomicAdd((unsigned long long *)&w.acc[0].pair[2], (unsigned long long)a2);
        atomicAdd((unsigned long long *)&w.acc[0].pair[3], (unsigned long long)a3);
    }
}

template <int KIND, int W>
static void launch_ccmc(int stage, const Work &w, const Grids &g, hipStream_t s)
{
    if (stage == 0) {
        k_ccmc_scan<W><<<256, CC_T, 0, s>>>(w);
        k_ccmc_clusters<KIND, W><<<g.ccmc, CC_T, 0, s>>>(w);
    } else {
        k_ccmc_singles<W><<<256, 256, 0, s>>>(w, stage == 2 ? 1 : 0);
        k_ccmc_pairs<KIND, W><<<64, 256, 0, s>>>(w);
    }
}

hipError_t enqueue_ccmc(int stage, int kind, const Work &w, const Grids &g, hipStream_t s)
{
    switch (kind * 16 + w.W) {
    case K_HUBBARD * 16 + 1: launch_ccmc<K_HUBBARD, 1>(stage, w, g, s); break;
    case K_UEG * 16 + 1: launch_ccmc<K_UEG, 1>(stage, w, g, s); break;
    case K_UEG * 16 + 2: launch_ccmc<K_UEG, 2>(stage, w, g, s); break;
    case K_UEG * 16 + 4: launch_ccmc<K_UEG, 4>(stage, w, g, s); break;
    case K_UEG * 16 + 8: launch_ccmc<K_UEG, 8>(stage, w, g, s); break;
    case K_MOLECULAR * 16 + 1: launch_ccmc<K_MOLECULAR, 1>(stage, w, g, s); break;
    case K_MOLECULAR * 16 + 2: launch_ccmc<K_MOLECULAR, 2>(stage, w, g, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fq
