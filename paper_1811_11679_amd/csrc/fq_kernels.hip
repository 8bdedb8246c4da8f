// Kernels of one FCIQMC projector iteration (paper Sec. 2.1 eq. fciqmc,
// Sec. 2.4 spawning / death / annihilation, appendix "Parallelization":
// sorted main list, spawned list sorted and merged into it), written for
// gfx950: 64-wide wavefronts, LDS-staged tiles, persistent grids that read
// their problem sizes from device memory, decoupled look-back for every
// prefix that crosses tiles (Merrill & Garland 2016) and a onesweep LSD
// radix sort (Adinets & Merrill 2022).
#include "fq_kernels.h"
#include "fq_scan.h"

#include <algorithm>

namespace fq {

// ---------------------------------------------------------------------------
// estimator accumulation. A thread sums its values in registers for one
// replica at a time; when it moves on to another replica (and at the end of
// the kernel) the values go to the block's table in LDS (replicas below
// acc_rows(R); others are added to global memory directly). At the end each
// block stores its table as one row of partials with plain stores and the
// iteration epilogue folds the rows. The accumulators are a few addresses
// that every block would otherwise hit with device-scope atomics.
// ---------------------------------------------------------------------------
struct LocalAcc {
    long long v[EST_FIELDS];
    int rep;
    __device__ void clear()
    {
#pragma unroll
        for (int i = 0; i < EST_FIELDS; ++i) v[i] = 0;
    }
};

__device__ __forceinline__ void acc_table_clear(long long *tab, int rl)
{
    for (int i = threadIdx.x; i < rl * EST_FIELDS; i += blockDim.x) tab[i] = 0;
}

__device__ __forceinline__ void acc_add(long long *tab, int rl, EstAcc *g, int rep, int f, long long v)
{
    if (rep < rl)
        atomicAdd((unsigned long long *)&tab[rep * EST_FIELDS + f], (unsigned long long)v);
    else
        atomicAdd((unsigned long long *)(&g[rep].nw + f), (unsigned long long)v);
}

// the thread's values to the block table, lane by lane
__device__ __forceinline__ void acc_spill(LocalAcc &a, long long *tab, int rl, EstAcc *g)
{
    if (a.rep < 0) return;
#pragma unroll
    for (int f = 0; f < EST_FIELDS; ++f)
        if (a.v[f]) acc_add(tab, rl, g, a.rep, f, a.v[f]);
    a.clear();
}

__device__ __forceinline__ void acc_switch(LocalAcc &acc, int rep, long long *tab, int rl, EstAcc *g)
{
    if (rep == acc.rep) return;
    acc_spill(acc, tab, rl, g);
    acc.rep = rep;
}

// end of a kernel (all threads): reduce over the wave when its active lanes
// hold one replica, then store the block's table as partial row blockIdx.x
__device__ void acc_finish(LocalAcc &a, bool active, long long *tab, int rl, EstAcc *g, long long *part)
{
    const uint64_t act = __ballot(active);
    if (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int rep0 = __shfl(a.rep, leader, 64);
        const bool uniform = __ballot(active && a.rep != rep0) == 0;
        if (uniform) {
#pragma unroll
            for (int f = 0; f < EST_FIELDS; ++f) {
                const long long sv = wave_sum<long long>(active ? a.v[f] : 0);
                if (lane_id() == leader && sv != 0) acc_add(tab, rl, g, rep0, f, sv);
            }
        } else if (active) {
            acc_spill(a, tab, rl, g);
        }
    }
    a.clear();
    __syncthreads();
    // partials are laid out [replica][field][block] so that the fold reads
    // each (replica, field) as one contiguous run
    for (int i = threadIdx.x; i < rl * EST_FIELDS; i += blockDim.x) part[(size_t)i * PART_MAX_BLOCKS + blockIdx.x] = tab[i];
}

enum { F_NW = 0, F_NOCC, F_N0, F_NSPAWN, F_NUNIQ, F_FLIPS, F_REJU, F_DEATH, F_SPAWN, F_REJ, F_L0, F_L1, F_L2, F_L3 };

// Time-step search maxima, per replica, into the replica's estimator record
// of the iteration: KD = false the largest |H_ji| / p_gen (as its bits), true
// the largest K_ii (as an order-preserving key). A thread keeps the running
// maximum of one replica and hands it over when it moves to another replica
// and at the end of the kernel; there the wave reduces first when its holders
// share one replica (the lists are sorted by replica, so they nearly always do).
template <bool KD>
__device__ __forceinline__ void ts_put(const Work &w, int rep, double v)
{
    if constexpr (KD)
        atomicMax(&w.acc[rep].kd_key, ordered_key(v));
    else
        atomicMax(&w.acc[rep].rs_bits, (unsigned long long)__double_as_longlong(v));
}

template <bool KD>
__device__ void ts_finish(const Work &w, double v, int rep, bool has)
{
    const uint64_t act = __ballot(has);
    if (!act) return;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int r0 = __shfl(rep, leader, 64);
    if (__ballot(has && rep != r0) == 0) {
        const double m = wave_max(has ? v : -INFINITY);
        if (lane_id() == leader) ts_put<KD>(w, r0, m);
    } else if (has) {
        ts_put<KD>(w, rep, v);
    }
}

// ---------------------------------------------------------------------------
// iteration prologue / epilogue
// ---------------------------------------------------------------------------
__global__ void k_begin(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        c->t += 1;
        c->n_main = c->n_main_new;
        c->n_spawn = 0;
        c->n_uniq = 0;
        c->n_att = c->n_att_new;
        c->collision = 0;
        c->ccmc_n0 = 0;
        c->ccmc_nex = 0;
        c->n_single = 0;
    }
    for (int i = threadIdx.x; i < TK_COUNT; i += blockDim.x) c->tickets[i] = 0;
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&c->hist[0][0])[i] = 0;
    for (int i = threadIdx.x; i < w.R * (int)(sizeof(EstAcc) / 8); i += blockDim.x) ((long long *)w.acc)[i] = 0;
}

__global__ __launch_bounds__(1024) void k_end(Work w, int nb_red, int nb_mrg)
{
    // one block per replica, one wave per estimator field: fold the partials
    // of the reduction and the merge into the accumulators, then record them
    // in the history ring
    const Ctl *c = w.ctl;
    if (c->err) return;
    const int r = blockIdx.x;
    const int f = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (r < acc_rows(w.R) && f < EST_FIELDS) {
        const long long *pr = w.part_red + (size_t)(r * EST_FIELDS + f) * PART_MAX_BLOCKS;
        const long long *pm = w.part_mrg + (size_t)(r * EST_FIELDS + f) * PART_MAX_BLOCKS;
        long long sum = 0;
        for (int b = lane; b < nb_red; b += 64) sum += pr[b];
        for (int b = lane; b < nb_mrg; b += 64) sum += pm[b];
        sum = wave_sum<long long>(sum);
        if (lane == 0) (&w.acc[r].nw)[f] += sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        EstAcc a = w.acc[r];
        a.t = c->t;
        w.hist[(size_t)(c->t % (uint32_t)w.hist_len) * w.R + r] = a;
    }
}

// ---------------------------------------------------------------------------
// attempt scan (set-up only; iterations get the prefix from the merge):
// att_off = exclusive prefix of natt over the main list
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

__global__ __launch_bounds__(SCAN_T) void k_scan_attempts(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    const long long n = c->n_main;
    const long long ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    const uint32_t epoch = epoch_of(c->t, 8);
    __shared__ long long s_tile, s_base;
    __shared__ long long s_red[8];
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[TK_SCAN], 1u);
        __syncthreads();
        const long long tile = s_tile;
        if (tile >= ntiles) break;
        const long long base = tile * SCAN_TILE + (long long)threadIdx.x * SCAN_I;
        long long v[SCAN_I];
        long long sum = 0;
#pragma unroll
        for (int i = 0; i < SCAN_I; ++i) {
            v[i] = (base + i < n) ? (long long)w.cur.natt[base + i] : 0;
            sum += v[i];
        }
        long long tot;
        const long long ex = block_excl_scan<long long>(sum, tot, s_red);
        if (threadIdx.x < 64) {
            const long long lb_ = lookback(w.st_scan, tile, epoch, tot);
            if (threadIdx.x == 0) s_base = lb_;
        }
        __syncthreads();
        long long run = s_base + ex;
#pragma unroll
        for (int i = 0; i < SCAN_I; ++i) {
            if (base + i < n) w.att_off[base + i] = run;
            run += v[i];
        }
        if (tile == ntiles - 1 && threadIdx.x == 0) {
            w.att_off[n] = s_base + tot;
            c->n_att_new = s_base + tot;
        }
        __syncthreads();
    }
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        w.att_off[0] = 0;
        c->n_att_new = 0;
    }
}

// ---------------------------------------------------------------------------
// spawning (Sec. 2.4): one thread per attempt, parents found through the
// attempt prefix (load balanced: a heavily populated determinant spreads its
// attempts over many threads and tiles). A tile of 1024 consecutive attempts
// finds its spawn count, reserves that many records with one atomic on the
// spawn counter and writes them contiguously. The records of different tiles
// land in completion order: the radix sort and the segmented sums downstream
// make the result independent of it (equal keys are summed as exact
// integers), and a tile never waits on another.
// ---------------------------------------------------------------------------


__device__ __forceinline__ long long upper_bound_ll(const long long *a, long long lo, long long hi, long long x)
{
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_spawn_partition(Work w, int span_len)
{
    const Ctl *c = w.ctl;
    if (c->err) return;
    const long long total = c->n_att, n = c->n_main;
    const long long nspans = (total + span_len - 1) / span_len;
    if (nspans + 1 > w.span_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&((Ctl *)c)->err, ERR_SPAWN_CAP);
        return;
    }
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s <= nspans;
         s += (long long)gridDim.x * blockDim.x) {
        if (s == nspans) {
            w.span_lo[s] = n > 0 ? n - 1 : 0;
        } else {
            w.span_lo[s] = upper_bound_ll(w.att_off, 0, n + 1, s * span_len) - 1;
        }
    }
}

// MULTI = false: a single replica (rb = 0), so the replica index is 0, its
// parameters are uniform over the grid and a determinant's hash is its sort key.
// LT (single-replica electron gas): the generator's small tables are staged in
// LDS; a compile-time choice, so that their loads are LDS loads.
//
// LDS per block: the attempt offsets of the tile's parents and the first
// SP_STAGE spawn records (written out coalesced); records beyond that, rare at
// the spawn rates of the method, go to global memory directly.
constexpr int SP_STAGE = 256;
template <int KIND, int W, bool MULTI, bool LT, int SP_I>
__global__ __launch_bounds__(SP_T) void k_spawn(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    constexpr int SPAN = SP_T * SP_I;
    constexpr int LCAP = SPAN + 2;
    __shared__ long long s_off[LCAP];
    __shared__ uint32_t s_cnt[SP_I][SP_T / 64];
    __shared__ long long s_tile, s_base;
    __shared__ uint32_t s_rrep[MULTI ? SP_STAGE : 1];  // replica of a staged record
    __shared__ uint64_t s_rkey[W][SP_STAGE];
    __shared__ int32_t s_ramp[SP_STAGE];
    __shared__ uint8_t s_rinit[SP_STAGE];
    const long long total = c->n_att;
    const long long nspans = (total + SPAN - 1) / SPAN;
    if (nspans + 1 > w.span_cap) return;
    const uint32_t t = c->t;
    const bool ss = c->ss_active != 0;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    // time-step search: the largest |H_ji| / p_gen of this thread's attempts
    // of replica rs_rep
    const bool ts = w.tau_search != 0;
    double rs_max = 0.0;
    int rs_rep = 0;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    UegTables lu = w.sys[w.rep[0].sys].u;
    const double *hb_tri = nullptr;  // heat-bath pair weights staged in LDS (LT, molecular)
    if constexpr (LT && KIND == K_MOLECULAR) {
        const DevSys &sy0 = w.sys[w.rep[0].sys];
        const int nso = sy0.n_so, ntri = nso * (nso - 1) / 2;
        double *tt = (double *)dyn_lds;
        for (int x = threadIdx.x; x < ntri; x += SP_T) {
            // x -> (P, Q), P < Q, row by row
            int P = 0, rem = x;
            while (rem >= nso - 1 - P) {
                rem -= nso - 1 - P;
                ++P;
            }
            tt[x] = sy0.hb_S[P * nso + P + 1 + rem];
        }
        hb_tri = tt;
    }
    if constexpr (LT && KIND == K_UEG) {
        const int M = lu.M, nv = w.sys[w.rep[0].sys].vlen, ng = lu.gdim * lu.gdim * lu.gdim;
        int32_t *tn = (int32_t *)dyn_lds;
        double *tv = (double *)(dyn_lds + ((4 * M + 15) & ~15));
        int16_t *tg = (int16_t *)((unsigned char *)tv + ((8 * nv + 15) & ~15));
        for (int i = threadIdx.x; i < M; i += SP_T) tn[i] = lu.npk[i];
        for (int i = threadIdx.x; i < nv; i += SP_T) tv[i] = lu.vtab[i];
        for (int i = threadIdx.x; i < ng; i += SP_T) tg[i] = lu.grid[i];
        lu.npk = tn;
        lu.vtab = tv;
        lu.grid = tg;
        lu.vx = nullptr;
    }
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[TK_SPAWN], 1u);
        __syncthreads();
        const long long span = s_tile;
        if (span >= nspans) break;
        const long long lo = w.span_lo[span];
        const long long hi = w.span_lo[span + 1];  // parent of the next tile's first attempt
        const long long len = hi - lo + 2;
        const bool staged = len <= LCAP;
        if (staged)
            for (long long i = threadIdx.x; i < len; i += SP_T) s_off[i] = w.att_off[lo + i];
        __syncthreads();
        bool has[SP_I];
        uint64_t child[SP_I][W];
        int32_t amp[SP_I];
        uint8_t init[SP_I];
        uint32_t rep[SP_I];
        // phase 1: the parent of each attempt (blocked: thread t takes attempts
        // 4t .. 4t+3 of the tile; one search finds the first parent, later
        // attempts advance from it), its first attempt and its attempt count
        long long pi[SP_I], pa0[SP_I], pnat[SP_I];
        {
            long long ip = -1;
#pragma unroll
            for (int it = 0; it < SP_I; ++it) {
                pi[it] = -1;
                pa0[it] = 0;
                pnat[it] = 1;
                const long long a = span * SPAN + (long long)threadIdx.x * SP_I + it;
                if (a < total) {
                    long long i;
                    if (staged) {
                        if (ip < 0) {
                            int l = 0, h = (int)len;
                            while (l < h) {
                                const int m = (l + h) >> 1;
                                if (s_off[m] <= a) l = m + 1; else h = m;
                            }
                            ip = lo + l - 1;
                        } else {
                            while (s_off[ip - lo + 1] <= a) ++ip;
                        }
                        i = ip;
                    } else {
                        i = upper_bound_ll(w.att_off, lo, hi + 2, a) - 1;
                    }
                    pi[it] = i;
                    pa0[it] = staged ? s_off[i - lo] : w.att_off[i];
                    pnat[it] = (staged ? s_off[i - lo + 1] : w.att_off[i + 1]) - pa0[it];
                }
            }
        }
        // phase 2 (short keys): every parent load of the thread in flight at once
        constexpr bool PF = W <= 2;
        uint64_t pkey[PF ? SP_I : 1][W];
        int32_t pn0[PF ? SP_I : 1], pdsl[PF ? SP_I : 1];
        uint64_t ppsk[PF ? SP_I : 1];
        if constexpr (PF) {
#pragma unroll
            for (int it = 0; it < SP_I; ++it) {
                const long long i = pi[it] < 0 ? 0 : pi[it];
#pragma unroll
                for (int q = 0; q < W; ++q) pkey[it][q] = w.cur.key[(size_t)q * w.main_cap + i];
                pn0[it] = w.cur.pop[i];
                pdsl[it] = ss ? w.cur.dslot[i] : -1;  // read only with the deterministic space active
                ppsk[it] = stored_skey(MULTI, W) ? w.cur.skey[i] : 0;
            }
        }
        // phase 3: excitation, matrix element, amplitude
#pragma unroll
        for (int it = 0; it < SP_I; ++it) {
            has[it] = false;
            amp[it] = 0;
            init[it] = 0;
            rep[it] = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) child[it][q] = 0;
            if (pi[it] >= 0) {
                const long long i = pi[it];
                const long long nat = pnat[it];
                const long long k = span * SPAN + (long long)threadIdx.x * SP_I + it - pa0[it];
                uint64_t key[W];
                int32_t n0, dsl;
                uint64_t psk;
                if constexpr (PF) {
#pragma unroll
                    for (int q = 0; q < W; ++q) key[q] = pkey[it][q];
                    n0 = pn0[it];
                    dsl = pdsl[it];
                    psk = ppsk[it];
                } else {
#pragma unroll
                    for (int q = 0; q < W; ++q) key[q] = w.cur.key[(size_t)q * w.main_cap + i];
                    n0 = w.cur.pop[i];
                    dsl = ss ? w.cur.dslot[i] : -1;
                    psk = stored_skey(MULTI, W) ? w.cur.skey[i] : 0;
                }
                rep[it] = MULTI ? skey_rep(psk, w.rb) : 0u;
                const RepParams &rp = w.rep[MULTI ? rep[it] : 0u];
                const DevSys &sy = w.sys[rp.sys];
                const uint64_t h = (!MULTI && W > 2) ? psk : hash64<W>(key);
                const long long an = n0 < 0 ? -(long long)n0 : (long long)n0;
                const bool pin_d = ss && dsl >= 0;
                // the determinant the generator acts on: the entry itself, or for
                // a pair (Sec. 2.3) the bra (even attempts of DMQMC) or the ket
                // (odd attempts of DMQMC; every attempt of IP-DMQMC)
                constexpr int BK = base_kind(KIND), WG = is_pair(KIND) ? W / 2 : W;
                int side = 0;
                long long nat_s = nat;  // attempts per end
                if constexpr (is_pair(KIND)) {
                    side = w.dm == 1 ? (int)(k & 1) : 1;
                    if (w.dm == 1) nat_s = nat >> 1;
                    init[it] = 1;  // no initiator rule on pairs
                } else {
                    init[it] = (uint8_t)(an > rp.thr || key_eq<W>(key, *(const uint64_t(*)[W])sy.ref) || pin_d);
                }
                uint64_t gdet[WG], gchild[WG];
#pragma unroll
                for (int q = 0; q < WG; ++q) {
                    gdet[q] = key[side * WG + q];
                    gchild[q] = 0;
                }
                const U4 r0 = draw(TAG_SELECT, (uint32_t)k, t, h, rp.k0, rp.k1);
                double pgen = 0.0, hv = 0.0;
                bool ok;
                if constexpr (BK == K_HUBBARD)
                    ok = gen_hubbard<WG>(sy, gdet, r0.x, gchild, pgen, hv);
                else if constexpr (BK == K_UEG)
                    ok = gen_ueg<WG>(LT ? lu : sy.u, gdet, r0.x, r0.y, gchild, pgen, hv);
                else
                    ok = gen_heatbath<WG>(sy, rp.p_single, gdet, r0, (uint32_t)k, t, h, rp.k0, rp.k1, gchild, pgen, hv,
                                          hb_tri);
#pragma unroll
                for (int q = 0; q < W; ++q) child[it][q] = key[q];
#pragma unroll
                for (int q = 0; q < WG; ++q) child[it][side * WG + q] = gchild[q];
                if (ok && hv != 0.0) {
                    bool skip = false;
                    if constexpr (!is_pair(KIND)) {
                        // CCMC: amplitudes exist only up to the truncation level
                        if (w.ccmc_trunc > 0) {
                            int d = 0;
#pragma unroll
                            for (int q = 0; q < W; ++q) d += __popcll(child[it][q] ^ sy.ref[q]);
                            skip = (d >> 1) > w.ccmc_trunc;
                        }
                    }
                    if (!skip && pin_d) {
                        // discard spawns that stay inside the deterministic space
                        const uint64_t cs = make_skey(hash64<W>(child[it]) & w.hmask, rep[it], w.rb);
                        const int nd = w.ds.n * w.R;
                        int l = 0, hh = nd;
                        while (l < hh) {
                            const int m = (l + hh) >> 1;
                            const uint64_t sk = w.ds.skey_sorted[m];
                            bool less = sk < cs;
                            if (sk == cs) {
                                uint64_t dk[W];
#pragma unroll
                                for (int q = 0; q < W; ++q) dk[q] = w.ds.key_sorted[(size_t)q * nd + m];
                                less = key_cmp<W>(dk, child[it]) < 0;
                            }
                            if (less) l = m + 1; else hh = m;
                        }
                        if (l < nd && w.ds.skey_sorted[l] == cs) {
                            uint64_t dk[W];
#pragma unroll
                            for (int q = 0; q < W; ++q) dk[q] = w.ds.key_sorted[(size_t)q * nd + l];
                            skip = key_eq<W>(dk, child[it]);
                        }
                    }
                    if (!skip) {
                        const double ah = fabs(hv);
                        if (ts) {
                            if (MULTI && (int)rep[it] != rs_rep) {
                                if (rs_max > 0.0) ts_put<false>(w, rs_rep, rs_max);
                                rs_max = 0.0;
                                rs_rep = (int)rep[it];
                            }
                            rs_max = fmax(rs_max, ah / pgen);
                        }
                        // DMQMC: the symmetrised Bloch equation's dbeta / 2 at each end
                        const double tau_s = (is_pair(KIND) && w.dm == 1) ? rp.tau * 0.5 : rp.tau;
                        double m;
                        if (rp.bits == 0)
                            m = (tau_s * ah) / pgen;
                        else if (nat_s == 1)
                            m = ((tau_s * ah) / pgen) * (double)an;  // x / 1.0 is x
                        else
                            m = (((tau_s * ah) / pgen) * (double)an) / (double)nat_s;
                        // the Hubbard and electron-gas generators leave the last two
                        // words of the selection block unused: they give the
                        // rounding uniform; heat-bath uses a block of its own
                        double u;
                        if constexpr (BK == K_MOLECULAR) {
                            const U4 rr = draw(TAG_SPAWN_ROUND, (uint32_t)k, t, h, rp.k0, rp.k1);
                            u = u53(rr.x, rr.y);
                        } else {
                            u = u53(r0.z, r0.w);
                        }
                        long long kk = 0;
                        if (!(m < 0x1p31)) {
                            atomicOr(&c->err, ERR_OVERFLOW);
                        } else {
                            if (rp.bits != 0 && m < (double)rp.cu)
                                kk = (u * (double)rp.cu < m) ? rp.cu : 0;
                            else
                                kk = sround(m, u);
                            if (kk > 2147483647ll) {
                                atomicOr(&c->err, ERR_OVERFLOW);
                                kk = 0;
                            }
                        }
                        if (kk != 0) {
                            const int sh = hv > 0.0 ? 1 : -1;
                            const int sn = n0 > 0 ? 1 : -1;
                            amp[it] = (int32_t)(-(long long)(sh * sn) * kk);
                            has[it] = true;
                        }
                    }
                }
            }
            const uint64_t m = __ballot(has[it]);
            if (lane == 0) s_cnt[it][wid] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        // offsets in attempt order: slab it, wave wid, lane
        uint32_t tot = 0, before[SP_I];
#pragma unroll
        for (int it = 0; it < SP_I; ++it)
#pragma unroll
            for (int q = 0; q < SP_T / 64; ++q) {
                if (q == wid) before[it] = tot;
                tot += s_cnt[it][q];
            }
        // the tile's output range, reserved with one atomic: records land in
        // tile completion order, which the sort and the segmented sums make
        // irrelevant (equal keys are summed as exact integers)
        if (threadIdx.x == 0) s_base = (long long)atomicAdd(&c->n_spawn, (unsigned long long)tot);
        // staged records get their sort key (a hash of the child) in the dense
        // output loop below, not in the divergent per-attempt code
        uint32_t rk[SP_I];
#pragma unroll
        for (int it = 0; it < SP_I; ++it) {
            const uint64_t m = __ballot(has[it]);
            rk[it] = before[it] + (uint32_t)__popcll(m & lanemask_lt());
            if (has[it]) {
                const uint32_t r = rk[it];
                if (r < SP_STAGE) {
                    if constexpr (MULTI) s_rrep[r] = rep[it];
#pragma unroll
                    for (int q = 0; q < W; ++q) s_rkey[q][r] = child[it][q];
                    s_ramp[r] = amp[it];
                    s_rinit[r] = init[it];
                }
            }
        }
        __syncthreads();
        const long long base = s_base;
        if (base + tot > w.spawn_cap) {
            if (threadIdx.x == 0) atomicOr(&c->err, ERR_SPAWN_CAP);
        } else {
            const uint32_t ns = tot < SP_STAGE ? tot : SP_STAGE;
            for (uint32_t p = threadIdx.x; p < ns; p += SP_T) {
                const long long o = base + p;
                uint64_t key[W];
#pragma unroll
                for (int q = 0; q < W; ++q) key[q] = s_rkey[q][p];
                w.sp.skey[o] = make_skey(hash64<W>(key) & w.hmask, MULTI ? s_rrep[p] : 0u, w.rb);
                uint64_t *rec = w.sp.rec + (size_t)o * (W + 1);
#pragma unroll
                for (int q = 0; q < W; ++q) rec[q] = key[q];
                rec[W] = (uint64_t)(uint32_t)s_ramp[p] | ((uint64_t)s_rinit[p] << 32);
            }
#pragma unroll
            for (int it = 0; it < SP_I; ++it)
                if (has[it] && rk[it] >= SP_STAGE) {
                    const long long o = base + rk[it];
                    w.sp.skey[o] = make_skey(hash64<W>(child[it]) & w.hmask, rep[it], w.rb);
                    uint64_t *rec = w.sp.rec + (size_t)o * (W + 1);
#pragma unroll
                    for (int q = 0; q < W; ++q) rec[q] = child[it][q];
                    rec[W] = (uint64_t)(uint32_t)amp[it] | ((uint64_t)init[it] << 32);
                }
        }
        __syncthreads();
    }
    if (ts) ts_finish<false>(w, rs_max, rs_rep, rs_max > 0.0);
}

// ---------------------------------------------------------------------------
// onesweep LSD radix sort of (sort key, index) pairs, 8 passes of 8 bits
// ---------------------------------------------------------------------------
// Tiles of 256 threads x OS_I keys: 2048 (8 per thread), 3072 (12: three
// blocks fit a compute unit's LDS) or 4096 (16), chosen per context
constexpr int OS_T = 256, OS_WAVES = OS_T / 64;
static_assert(SORT_TILE_MIN == 8 * OS_T, "the status words are sized for the smallest sort tile");

__global__ __launch_bounds__(256) void k_sort_hist(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    __shared__ uint32_t h[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const long long n = (long long)min(c->n_spawn, (unsigned long long)w.spawn_cap);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const uint64_t k = w.sp.skey[i];
#pragma unroll
        for (int p = 0; p < 8; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 255], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) {
        const uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&(&c->hist[0][0])[i], v);
    }
}

// predecessors a digit's look-back reads per round trip after the first (an
// instrumented copy measured ~12 round trips per walk at four; eight made
// each pass slower, the wider reads costing more than the shorter walks)
constexpr int SORT_LB = 4;

template <int OS_I>
__global__ __launch_bounds__(OS_T) void k_sort_pass(Work w, int pass, const uint64_t *kin, const uint32_t *iin,
                                                    uint64_t *kout, uint32_t *iout)
{
    constexpr int OS_TILE = OS_T * OS_I;
    Ctl *c = w.ctl;
    if (c->err) return;
    __shared__ uint64_t lk[OS_TILE];
    __shared__ uint32_t li[OS_TILE];
    __shared__ uint32_t wh[OS_WAVES][256];
    __shared__ uint32_t gofs[256];     // global digit start (from the histogram)
    __shared__ uint32_t lofs[256];     // digit start inside the tile
    __shared__ long long gbase[256];   // tile's first output per digit
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_red[8];
    const long long n = (long long)min(c->n_spawn, (unsigned long long)w.spawn_cap);
    const long long ntiles = (n + OS_TILE - 1) / OS_TILE;
    const uint32_t epoch = epoch_of(c->t, (uint32_t)pass);
    const int shift = 8 * pass;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    {
        // global exclusive digit offsets of this pass
        const uint32_t v = c->hist[pass][threadIdx.x];
        uint32_t tot;
        gofs[threadIdx.x] = block_excl_scan<uint32_t>(v, tot, s_red);
    }
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[TK_SORT + pass], 1u);
        __syncthreads();
        const long long tile = s_tile;
        if (tile >= ntiles) break;
        const long long tbase = tile * OS_TILE;
        const int tcount = (int)min((long long)OS_TILE, n - tbase);
        for (int i = threadIdx.x; i < OS_WAVES * 256; i += OS_T) (&wh[0][0])[i] = 0;
        __syncthreads();
        uint64_t kk[OS_I];
        uint32_t ix[OS_I];
        uint32_t rk[OS_I];
        // warp-striped sub-tile: element e = tbase + wid*64*OS_I + i*64 + lane
#pragma unroll
        for (int i = 0; i < OS_I; ++i) {
            const int le = wid * 64 * OS_I + i * 64 + lane;
            const long long e = tbase + le;
            const bool valid = le < tcount;
            kk[i] = valid ? kin[e] : 0;
            ix[i] = valid ? (iin ? iin[e] : (uint32_t)e) : 0;
            const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t m = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? m : ~m;
            }
            uint32_t r = 0;
            if (valid) r = wh[wid][d] + (uint32_t)__popcll(peers & lanemask_lt());
            __builtin_amdgcn_wave_barrier();
            if (valid && lane == __ffsll((unsigned long long)peers) - 1) wh[wid][d] += (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            rk[i] = r;
        }
        __syncthreads();
        {
            const int d = threadIdx.x;
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < OS_WAVES; ++q) {
                const uint32_t x = wh[q][d];
                wh[q][d] = run;
                run += x;
            }
            uint32_t tot;
            const uint32_t lo = block_excl_scan<uint32_t>(run, tot, s_red);
            lofs[d] = lo;
            gbase[d] = run;  // temporarily the tile count
        }
        __syncthreads();
        {
            const int d = threadIdx.x;
            const long long cnt = gbase[d];
            unsigned long long *st = w.st_sort + (size_t)tile * 256 + d;
            long long excl = 0;
            if (tile == 0) {
                st_store(st, st_pack(epoch, ST_INC, cnt));
            } else {
                st_store(st, st_pack(epoch, ST_AGG, cnt));
                long long j = tile - 1;
                int width = 1;  // the immediate predecessor first, then SORT_LB per round trip
                for (;;) {
                    unsigned long long s4[SORT_LB];
#pragma unroll
                    for (int u = 0; u < SORT_LB; ++u)
                        s4[u] = (u < width && j - u >= 0) ? st_load(w.st_sort + (size_t)(j - u) * 256 + d) : 0ull;
                    bool done = false, stop = false;
                    int used = 0;
                    long long add = 0;
#pragma unroll
                    for (int u = 0; u < SORT_LB; ++u) {
                        if (done || stop || u >= width) continue;
                        const unsigned long long s = s4[u];
                        const uint32_t e = (uint32_t)(s >> 40);
                        const unsigned long long f = (s >> ST_VBITS) & 3ull;
                        if (j - u < 0 || e != epoch || f == 0) {
                            stop = true;
                            continue;
                        }
                        add += (long long)(s & ST_VMASK);
                        ++used;
                        if (f == ST_INC) done = true;
                    }
                    excl += add;
                    j -= used;
                    if (done) break;
                    if (used == 0) __builtin_amdgcn_s_sleep(1);
                    width = SORT_LB;
                }
                st_store(st, st_pack(epoch, ST_INC, excl + cnt));
            }
            gbase[d] = (long long)gofs[d] + excl;
        }
        __syncthreads();
        // scatter into LDS in digit order (stable)
#pragma unroll
        for (int i = 0; i < OS_I; ++i) {
            const int le = wid * 64 * OS_I + i * 64 + lane;
            if (le < tcount) {
                const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
                const uint32_t pos = lofs[d] + wh[wid][d] + rk[i];
                lk[pos] = kk[i];
                li[pos] = ix[i];
            }
        }
        __syncthreads();
        for (int p = threadIdx.x; p < tcount; p += OS_T) {
            const uint64_t k = lk[p];
            const uint32_t d = (uint32_t)(k >> shift) & 255u;
            const long long o = gbase[d] + (p - (long long)lofs[d]);
            kout[o] = k;
            iout[o] = li[p];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// segmented reduction of the sorted spawned list (Sec. 2.4 annihilation:
// combine walkers on the same determinant): one entry per distinct
// determinant with the int64 sum of amplitudes and the OR of initiator flags
// ---------------------------------------------------------------------------
constexpr int RD_T = 256, RD_I = 4, RD_TILE = RD_T * RD_I;

template <int W>
__global__ __launch_bounds__(RD_T) void k_reduce(Work w, int second)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    if (second && !c->collision) return;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    long long *tab = (long long *)dyn_lds;  // estimator table, acc_rows(R) rows
    const int rl = acc_rows(w.R);
    acc_table_clear(tab, rl);
    __shared__ uint64_t s_lastk[RD_T][W];
    __shared__ uint64_t s_lasts[RD_T];
    __shared__ long long s_tile, s_base;
    __shared__ long long s_red[8];
    __shared__ long long s_ws[RD_T / 64];
    __shared__ uint32_t s_wf[RD_T / 64];
    __shared__ int s_wr[RD_T / 64];
    const long long n = (long long)min(c->n_spawn, (unsigned long long)w.spawn_cap);
    const long long ntiles = (n + RD_TILE - 1) / RD_TILE;
    const uint32_t epoch = epoch_of(c->t, second ? 10 : 9);
    const uint64_t *skey = w.sp.skey;
    const uint32_t *idx = w.sp.idx;
    LocalAcc acc;
    acc.clear();
    acc.rep = -1;
    bool any = false;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[second ? TK_RED2 : TK_RED1], 1u);
        __syncthreads();
        const long long tile = s_tile;
        if (tile >= ntiles) break;
        const long long base = tile * RD_TILE + (long long)threadIdx.x * RD_I;
        uint64_t sk[RD_I], kk[RD_I][W];
        int32_t am[RD_I];
        uint32_t fl[RD_I];
        bool valid[RD_I];
        bool head[RD_I];
        int nh = 0;
        // first pass with keys of up to two words: the tile's count goes out
        // before the gathers (below); otherwise after them
        constexpr bool SHORT = W <= 2;
        const bool early = SHORT && !second;
        long long ex = 0, tot = 0;
        if constexpr (SHORT) {
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                const long long e = base + i;
                valid[i] = e < n;
                sk[i] = valid[i] ? skey[e] : 0;
            }
            s_lasts[threadIdx.x] = sk[RD_I - 1];
            __syncthreads();
            const uint64_t psk0 = threadIdx.x > 0 ? s_lasts[threadIdx.x - 1] : (base > 0 ? skey[base - 1] : 0);
            // First pass, keys of up to two words: a segment starts wherever the
            // sort key changes (equal keys holding different determinants are a
            // collision, flagged below, after which the fix-up and the second pass
            // redo the tile). The tile's segment count then needs no record, so it
            // is published before the gathers, and the tiles after this one do not
            // wait on them. (Longer keys keep the single look-back after the
            // gathers: the early count would cost them a wave per SIMD.)
            if (early) {
                int nh0 = 0;
                uint64_t p = psk0;
                bool hp = base > 0;
#pragma unroll
                for (int i = 0; i < RD_I; ++i) {
                    if (valid[i]) nh0 += (hp && p == sk[i]) ? 0 : 1;
                    p = sk[i];
                    hp = true;
                }
                ex = block_excl_scan<long long>((long long)nh0, tot, s_red);
                if (threadIdx.x == 0) lookback_publish(w.st_red, tile, epoch, tot);
            }
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                am[i] = 0;
                fl[i] = 0;
#pragma unroll
                for (int q = 0; q < W; ++q) kk[i][q] = 0;
                if (valid[i]) {
                    const uint64_t *rec = w.sp.rec + (size_t)idx[base + i] * (W + 1);
#pragma unroll
                    for (int q = 0; q < W; ++q) kk[i][q] = rec[q];
                    const uint64_t ai = rec[W];
                    am[i] = (int32_t)(uint32_t)ai;
                    fl[i] = (uint32_t)(ai >> 32);
                }
            }
#pragma unroll
            for (int q = 0; q < W; ++q) s_lastk[threadIdx.x][q] = kk[RD_I - 1][q];
            __syncthreads();
            uint64_t psk = psk0;
            uint64_t pk[W];
            bool have_prev = base > 0;
            if (threadIdx.x > 0) {
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = s_lastk[threadIdx.x - 1][q];
            } else if (base > 0) {
                const uint64_t *rec = w.sp.rec + (size_t)idx[base - 1] * (W + 1);
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = rec[q];
            } else {
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = 0;
            }
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                head[i] = false;
                if (valid[i]) {
                    const bool same_s = have_prev && psk == sk[i];
                    const bool same_k = same_s && key_eq<W>(pk, kk[i]);
                    if (same_s && !same_k) atomicOr(&c->collision, 1u);
                    // the second pass follows the key order the fix-up gave each
                    // collision run
                    head[i] = early ? !same_s : !same_k;
                    nh += head[i];
                }
                psk = sk[i];
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = kk[i][q];
                have_prev = true;
            }
        } else {
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                const long long e = base + i;
                valid[i] = e < n;
                sk[i] = 0;
                am[i] = 0;
                fl[i] = 0;
#pragma unroll
                for (int q = 0; q < W; ++q) kk[i][q] = 0;
                if (valid[i]) {
                    sk[i] = skey[e];
                    const uint64_t *rec = w.sp.rec + (size_t)idx[e] * (W + 1);
#pragma unroll
                    for (int q = 0; q < W; ++q) kk[i][q] = rec[q];
                    const uint64_t ai = rec[W];
                    am[i] = (int32_t)(uint32_t)ai;
                    fl[i] = (uint32_t)(ai >> 32);
                }
            }
            s_lasts[threadIdx.x] = sk[RD_I - 1];
#pragma unroll
            for (int q = 0; q < W; ++q) s_lastk[threadIdx.x][q] = kk[RD_I - 1][q];
            __syncthreads();
            uint64_t psk;
            uint64_t pk[W];
            bool have_prev = base > 0;
            if (threadIdx.x > 0) {
                psk = s_lasts[threadIdx.x - 1];
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = s_lastk[threadIdx.x - 1][q];
            } else if (base > 0) {
                psk = skey[base - 1];
                const uint64_t *rec = w.sp.rec + (size_t)idx[base - 1] * (W + 1);
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = rec[q];
            } else {
                psk = 0;
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = 0;
            }
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                head[i] = false;
                if (valid[i]) {
                    const bool same_s = have_prev && psk == sk[i];
                    const bool same_k = same_s && key_eq<W>(pk, kk[i]);
                    if (same_s && !same_k) atomicOr(&c->collision, 1u);
                    head[i] = !same_k;
                    nh += head[i];
                }
                psk = sk[i];
#pragma unroll
                for (int q = 0; q < W; ++q) pk[q] = kk[i][q];
                have_prev = true;
            }
        }
        // the open segment at this thread's end (after its last head, or all
        // of its elements without a head), passed to the right
        long long lead_s = 0, tail_s = 0;
        uint32_t lead_f = 0, tail_f = 0;
        {
            bool seen = false;
#pragma unroll
            for (int i = 0; i < RD_I; ++i) {
                if (!valid[i]) continue;
                if (head[i]) {
                    seen = true;
                    tail_s = 0;
                    tail_f = 0;
                }
                if (seen) {
                    tail_s += am[i];
                    tail_f |= fl[i];
                } else {
                    lead_s += am[i];
                    lead_f |= fl[i];
                }
            }
        }
        // exclusive segmented scan over the tile's threads: the partial sum and
        // flags of the segment open at this thread's first element (threads
        // with a head restart it)
        long long carry_s;
        uint32_t carry_f;
        {
            const int lane = lane_id(), wid = threadIdx.x >> 6;
            bool r = nh > 0;
            long long xs = r ? tail_s : lead_s;
            uint32_t xf = r ? tail_f : lead_f;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const long long ys = __shfl_up(xs, o, 64);
                const uint32_t yf = __shfl_up(xf, o, 64);
                const bool yr = __shfl_up((int)r, o, 64) != 0;
                if (lane >= o && !r) {
                    xs += ys;
                    xf |= yf;
                    r = yr;
                }
            }
            // wave totals, then the prefix of the earlier waves
            if (lane == 63) {
                s_ws[wid] = xs;
                s_wf[wid] = xf;
                s_wr[wid] = r ? 1 : 0;
            }
            long long es = __shfl_up(xs, 1, 64);
            uint32_t ef = __shfl_up(xf, 1, 64);
            bool er = __shfl_up((int)r, 1, 64) != 0;
            if (lane == 0) {
                es = 0;
                ef = 0;
                er = false;
            }
            __syncthreads();
            if (!er) {
                long long ps = 0;
                uint32_t pf = 0;
                for (int q = 0; q < wid; ++q) {
                    if (s_wr[q]) {
                        ps = 0;
                        pf = 0;
                    }
                    ps += s_ws[q];
                    pf |= s_wf[q];
                }
                es += ps;
                ef |= pf;
            }
            carry_s = es;
            carry_f = ef;
        }
        if (!early) ex = block_excl_scan<long long>((long long)nh, tot, s_red);
        if (threadIdx.x < 64) {
            const long long lb_ = early ? lookback_wait(w.st_red, tile, epoch, tot) : lookback(w.st_red, tile, epoch, tot);
            if (threadIdx.x == 0) s_base = lb_;
        }
        __syncthreads();
        // Segment totals. A segment is stored by the thread holding its last
        // element in the tile: the thread of the next head, or the thread of
        // the tile's last element. The part of a segment whose head lies in an
        // earlier tile becomes this tile's boundary part.
        const long long tile_end = min(tile * RD_TILE + RD_TILE, n);
        long long seg = s_base + ex - 1;  // segment open at this thread's first element
        long long run_s = carry_s;
        uint32_t run_f = carry_f;
        bool run_here = ex > 0;  // its head is in this tile
        // whether the open segment holds elements of this tile before this thread
        bool run_nonempty = threadIdx.x > 0;
        BoundaryPart bp;
        bp.sum = 0;
        bp.seg = 0;
        bp.flag = 0;
        bp.valid = 0;
        bp.pad = 0;
        bool bp_mine = false;
        if (threadIdx.x == 0 && valid[0] && head[0]) bp_mine = true;  // no boundary part: record it as such
#pragma unroll
        for (int i = 0; i < RD_I; ++i) {
            if (!valid[i]) continue;
            if (head[i]) {
                if (run_nonempty) {
                    if (run_here) {
                        w.u.sum[seg] = run_s;
                        w.u.flag[seg] = run_f;
                    } else {
                        bp.sum = run_s;
                        bp.flag = run_f;
                        bp.seg = s_base - 1;
                        bp.valid = 1;
                        bp_mine = true;
                    }
                }
                ++seg;
                w.u.skey[seg] = sk[i];
#pragma unroll
                for (int q = 0; q < W; ++q) w.u.key[(size_t)q * w.spawn_cap + seg] = kk[i][q];
                run_s = 0;
                run_f = 0;
                run_here = true;
            }
            run_s += am[i];
            run_f |= fl[i];
            run_nonempty = true;
            if (base + i == tile_end - 1) {
                // the tile's last element closes its open segment here
                if (run_here) {
                    w.u.sum[seg] = run_s;
                    w.u.flag[seg] = run_f;
                } else {
                    bp.sum = run_s;
                    bp.flag = run_f;
                    bp.seg = s_base - 1;
                    bp.valid = 1;
                    bp_mine = true;
                }
            }
            acc_switch(acc, (int)skey_rep(sk[i], w.rb), tab, rl, w.acc);
            acc.v[F_NSPAWN] += 1;
            acc.v[F_SPAWN] += am[i];
            acc.v[F_NUNIQ] += head[i] ? 1 : 0;
            any = true;
        }
        if (bp_mine) w.bpart[tile] = bp;
        if (tile == ntiles - 1 && threadIdx.x == 0) c->n_uniq = s_base + tot;
        __syncthreads();
    }
    acc_finish(acc, any && acc.rep >= 0, tab, rl, w.acc, w.part_red);
}

// Rare path: equal sort keys holding different determinants (hash
// collisions) are put in key order and the reduction is redone. A run of
// equal sort keys can be long, since a determinant may receive many spawns:
// it is only reordered when it holds more than one determinant, by moving the
// entries of its smallest remaining determinant to the front, one determinant
// at a time (stable; run length x distinct determinants gathers, through the
// radix sort's ping-pong index buffer, which is free at this point).
constexpr int FIXUP_MAX_KEYS = 64;

template <int W>
__device__ __forceinline__ void rec_key(const Work &w, uint32_t j, uint64_t (&k)[W])
{
#pragma unroll
    for (int q = 0; q < W; ++q) k[q] = w.sp.rec[(size_t)j * (W + 1) + q];
}

template <int W>
__global__ void k_fixup(Work w)
{
    Ctl *c = w.ctl;
    if (c->err || !c->collision) return;
    const long long n = (long long)min(c->n_spawn, (unsigned long long)w.spawn_cap);
    const uint64_t *skey = w.sp.skey;
    uint32_t *idx = w.sp.idx;
    uint32_t *tmp = w.sp.idx2;
    const long long gs = (long long)gridDim.x * blockDim.x;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < w.R * (int)(sizeof(EstAcc) / 8); i += blockDim.x) {
            const int r = i / (int)(sizeof(EstAcc) / 8), f = i % (int)(sizeof(EstAcc) / 8);
            if (f == F_NSPAWN || f == F_NUNIQ || f == F_SPAWN) ((long long *)&w.acc[r])[f] = 0;
        }
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
        if (i > 0 && skey[i - 1] == skey[i]) continue;
        uint64_t k0[W];
        rec_key<W>(w, idx[i], k0);
        long long e = i + 1;
        bool mixed = false;
        while (e < n && skey[e] == skey[i]) {
            if (!mixed) {
                uint64_t ke[W];
                rec_key<W>(w, idx[e], ke);
                mixed = !key_eq<W>(ke, k0);
            }
            ++e;
        }
        if (!mixed) continue;
        for (long long a = i; a < e; ++a) tmp[a] = idx[a];
        long long pos = i;
        uint64_t prev[W];
        for (int d = 0;; ++d) {
            // the smallest determinant of the run above the last one placed
            bool found = false;
            uint64_t best[W];
            for (long long a = i; a < e; ++a) {
                uint64_t ka[W];
                rec_key<W>(w, tmp[a], ka);
                if (d > 0 && key_cmp<W>(ka, prev) <= 0) continue;
                if (!found || key_cmp<W>(ka, best) < 0) {
#pragma unroll
                    for (int q = 0; q < W; ++q) best[q] = ka[q];
                    found = true;
                }
            }
            if (!found) break;
            if (d == FIXUP_MAX_KEYS) {
                // this many determinants on one sort key cannot come from hash collisions
                atomicOr(&c->err, ERR_COLLISION);
                break;
            }
            for (long long a = i; a < e; ++a) {
                uint64_t ka[W];
                rec_key<W>(w, tmp[a], ka);
                if (key_eq<W>(ka, best)) idx[pos++] = tmp[a];
            }
#pragma unroll
            for (int q = 0; q < W; ++q) prev[q] = best[q];
        }
    }
}

// ---------------------------------------------------------------------------
// annihilation merge (Sec. 2.4; appendix "Parallelization"): merge-path merge
// of the distinct spawned determinants into the sorted main list, fused with
// death/cloning of existing entries, the deterministic-space update, the
// initiator rule for new determinants (Sec. 2.1), removal of empty entries,
// the estimators of the new list (tutorial appendix) and the attempt counts of
// the next iteration. Ties in the merge order put the main entry first.
//
// A tile's slices of both lists are staged in LDS with coalesced loads (main
// entries in slots [0, la), spawned ones in [la, la + lb)); every thread
// merges its run of positions from LDS, writes each result into the source
// slot, and the kept entries leave in merge order with coalesced stores.
// ---------------------------------------------------------------------------
// Keys of up to two words: 512 threads of two positions each, whose tile's
// dependent phases (ticket, partition, staging, look-back) are shorter than
// with 256 threads of four; two such blocks fit a compute unit's registers
// and LDS. Longer keys: 256 threads of two positions (their LDS slice is
// larger, and three such blocks per compute unit measured faster).
// MI: merge positions per thread and tile, 1, 2 or 4 for keys of up to two
// words (chosen per context), 2 for longer keys
template <int W, int MI>
struct MergeCfg {
    static constexpr int T = W <= 2 ? 512 : 256;
    static constexpr int I = MI;
    static constexpr int TILE = T * I;
};
static_assert(MergeCfg<1, 1>::TILE == 512 && MergeCfg<8, 2>::TILE == 512,
              "the merge partition and status arrays are sized for 512-position tiles");

template <int W>
__device__ __forceinline__ void load_key(const uint64_t *base, long long cap, long long i, uint64_t (&k)[W])
{
#pragma unroll
    for (int q = 0; q < W; ++q) k[q] = base[(size_t)q * cap + i];
}

// sort key of main entry i (see stored_skey)
template <int W>
__device__ __forceinline__ uint64_t main_skey(const Work &w, long long i)
{
    if (stored_skey(w.rb != 0, W)) return w.cur.skey[i];
    uint64_t k[W];
    load_key<W>(w.cur.key, w.main_cap, i, k);
    return hash64<W>(k);
}

// main[i] <= uniq[j] in (sort key, key) order (global memory)
template <int W>
__device__ __forceinline__ bool le_ab(const Work &w, long long i, uint64_t si, long long j, uint64_t sj)
{
    if (si != sj) return si < sj;
    uint64_t a[W], b[W];
    load_key<W>(w.cur.key, w.main_cap, i, a);
    load_key<W>(w.u.key, w.spawn_cap, j, b);
    return key_cmp<W>(a, b) <= 0;
}

template <int W, int MI>
__global__ void k_merge_partition(Work w)
{
    const Ctl *c = w.ctl;
    if (c->err) return;
    {
        // the segmented reduction's boundary parts (one per reduction tile at
        // most): the last reduction launch of the iteration has finished
        const long long ns = (long long)min(c->n_spawn, (unsigned long long)w.spawn_cap);
        const long long nrt = (ns + RD_TILE - 1) / RD_TILE;
        for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nrt; t += (long long)gridDim.x * blockDim.x) {
            const BoundaryPart b = w.bpart[t];
            if (b.valid) {
                atomicAdd((unsigned long long *)&w.u.sum[b.seg], (unsigned long long)b.sum);
                if (b.flag) atomicOr(&w.u.flag[b.seg], b.flag);
            }
        }
    }
    constexpr int TILE = MergeCfg<W, MI>::TILE;
    const long long na = c->n_main, nb = c->n_uniq;
    const long long ntiles = (na + nb + TILE - 1) / TILE;
    for (long long tile = (long long)blockIdx.x * blockDim.x + threadIdx.x; tile <= ntiles;
         tile += (long long)gridDim.x * blockDim.x) {
        const long long d = min(tile * TILE, na + nb);
        long long lo = max(0ll, d - nb), hi = min(d, na);
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            const long long j = d - 1 - mid;
            if (le_ab<W>(w, mid, main_skey<W>(w, mid), j, w.u.skey[j])) lo = mid + 1; else hi = mid;
        }
        w.mpart[tile] = lo;
    }
}


__device__ __forceinline__ void add_limbs(long long (&v)[EST_FIELDS], double x)
{
    add_limbs4(v[F_L0], v[F_L1], v[F_L2], v[F_L3], x);
}

// The value sum_k a_k 2^(32k - 64) of four limb sums, rounded once to the
// nearest FP64 value (ties to even).
__device__ double limbs_to_double(long long a0, long long a1, long long a2, long long a3)
{
    // signed 128-bit total as (hi, lo), two's complement
    uint64_t lo = 0, hi = 0;
    auto add_shifted = [&](long long v, int s) {
        // v * 2^s, s in {0, 32, 64, 96}, sign-extended to 128 bits
        const uint64_t ext = v < 0 ? ~0ull : 0ull;
        uint64_t vlo, vhi;
        if (s == 0) { vlo = (uint64_t)v; vhi = ext; }
        else if (s < 64) { vlo = (uint64_t)v << s; vhi = (ext << s) | ((uint64_t)v >> (64 - s)); }
        else if (s == 64) { vlo = 0; vhi = (uint64_t)v; }
        else { vlo = 0; vhi = (uint64_t)v << (s - 64); }
        const uint64_t nlo = lo + vlo;
        hi = hi + vhi + (nlo < lo ? 1ull : 0ull);
        lo = nlo;
    };
    add_shifted(a0, 0);
    add_shifted(a1, 32);
    add_shifted(a2, 64);
    add_shifted(a3, 96);
    if ((hi | lo) == 0) return 0.0;
    const bool neg = (long long)hi < 0;
    if (neg) {
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0 ? 1ull : 0ull);
    }
    // leading bit position of the magnitude
    const int msb = hi ? 127 - __clzll(hi) : 63 - __clzll(lo);
    double r;
    if (msb < 53) {
        r = (double)lo;  // exact
    } else {
        const int shift = msb - 52;  // bits below the 53-bit mantissa
        uint64_t m, rem_hi_bit, rem_rest;
        // m = magnitude >> shift; the dropped bits decide the rounding
        if (shift >= 64) {
            m = hi >> (shift - 64);
            const int rs = shift - 64;  // dropped bits of hi below m, then all of lo
            const uint64_t dh = rs ? (hi & ((1ull << rs) - 1)) : 0ull;
            rem_hi_bit = rs ? (dh >> (rs - 1)) & 1ull : (lo >> 63);
            rem_rest = rs ? ((dh & ((1ull << (rs - 1)) - 1)) | lo) : (lo & ~(1ull << 63));
        } else {
            m = (lo >> shift) | (shift ? hi << (64 - shift) : 0ull);
            const uint64_t dl = lo & ((1ull << shift) - 1);  // shift >= 1 here
            rem_hi_bit = (dl >> (shift - 1)) & 1ull;
            rem_rest = dl & ((1ull << (shift - 1)) - 1);
        }
        if (rem_hi_bit && (rem_rest || (m & 1ull))) m += 1;
        r = ldexp((double)m, shift);  // m <= 2^53: exact
    }
    r = r * 0x1p-64;
    return neg ? -r : r;
}

// spawning attempts of an entry holding p units: |p| for integer walkers,
// ceil(|p| 2^-b) for fixed point, times mult (2 for DMQMC pairs: that many
// at each end); 2^28 or more does not fit the counter's attempt field
__device__ __forceinline__ long long attempts_of(long long p, int bits, int mult, Ctl *c)
{
    const long long ap = p < 0 ? -p : p;
    const long long n = mult * (bits == 0 ? ap : (ap + (1ll << bits) - 1) >> bits);
    if (n >= (1ll << 28)) atomicOr(&c->err, ERR_ATTEMPTS);
    return n;
}

template <int KIND, int W, bool MULTI, int MI>
__global__ __launch_bounds__((MergeCfg<W, MI>::T)) void k_merge(Work w)
{
    Ctl *c = w.ctl;
    if (c->err) return;
    constexpr int MG_T = MergeCfg<W, MI>::T, TILE = MergeCfg<W, MI>::TILE;
    __shared__ uint64_t s_sk[TILE];
    __shared__ uint64_t s_key[W][TILE];
    __shared__ long long s_val[TILE];   // main: population, then the new one; spawned: sum
    __shared__ double s_kd[TILE];       // K_ii - H_00
    __shared__ int32_t s_meta[TILE];    // main: dslot; spawned: initiator flag, then dslot (-1)
    __shared__ uint16_t s_src[TILE];    // merge position -> slot
    __shared__ uint16_t s_dst[TILE];    // merge position -> rank among kept
    __shared__ uint8_t s_keep[TILE];
    __shared__ uint64_t s_pa_sk, s_pa_key[W];  // main entry before the tile
    __shared__ uint64_t s_nb_sk, s_nb_key[W];  // spawned entry after the tile
    __shared__ long long s_nb_sum;
    __shared__ int s_pa_ok, s_nb_ok;
    __shared__ long long s_tile, s_base, s_abase;
    __shared__ long long s_red[16];
    const long long na = c->n_main, nb = c->n_uniq;
    const long long ntiles = (na + nb + TILE - 1) / TILE;
    const uint32_t t = c->t;
    const uint32_t epoch = epoch_of(t, 11), epoch_att = epoch_of(t, 13);
    const bool ss = c->ss_active != 0;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    long long *tab = (long long *)dyn_lds;  // estimator table, acc_rows(R) rows
    const int rl = acc_rows(w.R);
    acc_table_clear(tab, rl);
    LocalAcc acc;
    acc.clear();
    acc.rep = -1;
    bool any = false;
    // time-step search: the largest K_ii of the entries this thread's death steps act on
    const bool ts = w.tau_search != 0;
    double kd_max = -INFINITY;
    int kd_rep = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tickets[TK_MERGE], 1u);
        __syncthreads();
        const long long tile = s_tile;
        if (tile >= ntiles) break;
        const long long d0 = tile * TILE, d1 = min(d0 + TILE, na + nb);
        const long long i0 = w.mpart[tile], i1 = w.mpart[tile + 1];
        const long long j0 = d0 - i0, j1 = d1 - i1;
        const int la = (int)(i1 - i0), lb = (int)(j1 - j0);
        for (int q = threadIdx.x; q < la; q += MG_T) {
            const long long g = i0 + q;
            uint64_t k[W];
#pragma unroll
            for (int x = 0; x < W; ++x) {
                k[x] = w.cur.key[(size_t)x * w.main_cap + g];
                s_key[x][q] = k[x];
            }
            s_sk[q] = stored_skey(MULTI, W) ? w.cur.skey[g] : hash64<W>(k);
            s_val[q] = w.cur.pop[g];
            s_kd[q] = w.cur.kdiag[g];
            s_meta[q] = ss ? w.cur.dslot[g] : -1;
        }
        for (int q = threadIdx.x; q < lb; q += MG_T) {
            const long long g = j0 + q;
            s_sk[la + q] = w.u.skey[g];
#pragma unroll
            for (int x = 0; x < W; ++x) s_key[x][la + q] = w.u.key[(size_t)x * w.spawn_cap + g];
            s_val[la + q] = w.u.sum[g];
            s_meta[la + q] = (int32_t)w.u.flag[g];
        }
        if (threadIdx.x == 0) {
            s_pa_ok = i0 > 0;
            if (i0 > 0) {
#pragma unroll
                for (int x = 0; x < W; ++x) s_pa_key[x] = w.cur.key[(size_t)x * w.main_cap + i0 - 1];
                s_pa_sk = stored_skey(MULTI, W) ? w.cur.skey[i0 - 1] : hash64<W>(s_pa_key);
            }
            s_nb_ok = j1 < nb;
            if (j1 < nb) {
                s_nb_sk = w.u.skey[j1];
#pragma unroll
                for (int x = 0; x < W; ++x) s_nb_key[x] = w.u.key[(size_t)x * w.spawn_cap + j1];
                s_nb_sum = w.u.sum[j1];
            }
        }
        __syncthreads();
        auto le = [&](int a, int b) -> bool {  // A slot a <= B slot la + b
            const uint64_t sa = s_sk[a], sb = s_sk[la + b];
            if (sa != sb) return sa < sb;
            int r = 0;
#pragma unroll
            for (int x = W - 1; x >= 0; --x)
                if (r == 0) r = s_key[x][a] < s_key[x][la + b] ? -1 : (s_key[x][a] > s_key[x][la + b] ? 1 : 0);
            return r <= 0;
        };
        auto eq_slots = [&](int p, int q) -> bool {
            bool e = s_sk[p] == s_sk[q];
#pragma unroll
            for (int x = 0; x < W; ++x) e = e && s_key[x][p] == s_key[x][q];
            return e;
        };
        const int dl = min((int)threadIdx.x * MI, la + lb);
        int lo = max(0, dl - lb), hi = min(dl, la);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (le(mid, dl - 1 - mid)) lo = mid + 1; else hi = mid;
        }
        int ia = lo, jb = dl - lo;
        const int steps = min(MI, la + lb - dl);
        for (int st = 0; st < steps; ++st) {
            const int m = dl + st;
            bool takeA;
            if (ia >= la) takeA = false;
            else if (jb >= lb) takeA = true;
            else takeA = le(ia, jb);
            if (takeA) {
                const int a = ia++;
                const uint64_t sk = s_sk[a];
                const int32_t n0 = (int32_t)s_val[a];
                const int32_t dsl = s_meta[a];
                const int rep = MULTI ? (int)skey_rep(sk, w.rb) : 0;
                acc_switch(acc, rep, tab, rl, w.acc);
                any = true;
                // matching spawned determinant: the next unconsumed one
                long long add = 0;
                if (jb < lb) {
                    if (eq_slots(a, la + jb)) add = s_val[la + jb];
                } else if (s_nb_ok && s_nb_sk == sk) {
                    bool e = true;
#pragma unroll
                    for (int x = 0; x < W; ++x) e = e && s_nb_key[x] == s_key[x][a];
                    if (e) add = s_nb_sum;
                }
                long long v;
                if (ss && dsl >= 0) {
                    v = (long long)n0 + w.ds.delta[(size_t)rep * w.ds.n + dsl];
                } else if (n0 != 0) {
                    const RepParams &rp = w.rep[rep];
                    if (ts) {
                        if (MULTI && rep != kd_rep) {
                            if (kd_max > -INFINITY) ts_put<true>(w, kd_rep, kd_max);
                            kd_max = -INFINITY;
                            kd_rep = rep;
                        }
                        kd_max = fmax(kd_max, s_kd[a]);
                    }
                    const double an = (double)(n0 < 0 ? -(long long)n0 : (long long)n0);
                    const double mm = (rp.tau * (s_kd[a] - w.shift[rep])) * an;
                    uint64_t h = sk;
                    if constexpr (MULTI) {
                        uint64_t key[W];
#pragma unroll
                        for (int x = 0; x < W; ++x) key[x] = s_key[x][a];
                        h = hash64<W>(key);
                    }
                    const U4 r = draw(TAG_DEATH, 0, t, h, rp.k0, rp.k1);
                    const double u = u53(r.x, r.y);
                    if (!(fabs(mm) < 0x1p40)) atomicOr(&c->err, ERR_OVERFLOW);
                    const long long k = mm >= 0.0 ? sround(mm, u) : -sround(-mm, u);
                    const long long sg = n0 > 0 ? 1 : -1;
                    v = (long long)n0 - sg * k;
                    if ((v > 0 && n0 < 0) || (v < 0 && n0 > 0)) acc.v[F_FLIPS] += 1;
                } else {
                    v = 0;
                }
                acc.v[F_DEATH] += v;
                v += add;
                if (v > 2147483647ll || v < -2147483647ll) atomicOr(&c->err, ERR_OVERFLOW);
                s_val[a] = v;
                s_src[m] = (uint16_t)a;
                s_keep[m] = (v != 0 || dsl >= 0) ? 1 : 0;
            } else {
                const int b = jb++;
                const int slot = la + b;
                // matched with the preceding main entry: that entry's thread added it
                bool matched;
                if (ia > 0) {
                    matched = eq_slots(ia - 1, slot);
                } else {
                    matched = s_pa_ok && s_pa_sk == s_sk[slot];
#pragma unroll
                    for (int x = 0; x < W; ++x) matched = matched && s_pa_key[x] == s_key[x][slot];
                }
                s_src[m] = (uint16_t)slot;
                s_keep[m] = 0;
                if (!matched) {
                    const long long sum = s_val[slot];
                    const int32_t fl = s_meta[slot];
                    const int rep = MULTI ? (int)skey_rep(s_sk[slot], w.rb) : 0;
                    const RepParams &rp = w.rep[rep];
                    acc_switch(acc, rep, tab, rl, w.acc);
                    any = true;
                    const bool accept = (!rp.initiator || fl) && sum != 0;
                    if (accept) {
                        if (sum > 2147483647ll || sum < -2147483647ll) atomicOr(&c->err, ERR_OVERFLOW);
                        // K_jj - H_00 is filled in by k_new_diag (off the merge's critical path)
                        s_kd[slot] = __longlong_as_double(0x7FF8000000000000ll);
                        s_meta[slot] = -1;
                        s_keep[m] = 1;
                    } else {
                        acc.v[F_REJU] += sum < 0 ? -sum : sum;
                        acc.v[F_REJ] += sum;
                    }
                }
            }
        }
        // ranks of the kept entries in merge order, and their spawning attempts
        // for the next iteration (the attempt prefix replaces a separate scan)
        int cnt = 0;
        long long asum = 0;
        for (int st = 0; st < steps; ++st) {
            const int m = dl + st;
            if (!s_keep[m]) continue;
            ++cnt;
            const int slot = s_src[m];
            const int rep = MULTI ? (int)skey_rep(s_sk[slot], w.rb) : 0;
            asum += attempts_of(s_val[slot], w.rep[rep].bits, w.dm == 1 ? 2 : 1, c);
        }
        long long tot, atot, ex, aex;
        block_excl_scan2((long long)cnt, asum, ex, aex, tot, atot, s_red);
        if (threadIdx.x < 64) {
            const long long lb_ = lookback(w.st_merge, tile, epoch, tot);
            if (threadIdx.x == 0) s_base = lb_;
        } else if (threadIdx.x < 128) {
            const long long lb_ = lookback(w.st_att, tile, epoch_att, atot);
            if (threadIdx.x == 64) s_abase = lb_;
        }
        {
            int r = (int)ex;
            for (int st = 0; st < steps; ++st)
                if (s_keep[dl + st]) s_dst[dl + st] = (uint16_t)r++;
        }
        __syncthreads();
        if (s_base + tot <= w.main_cap) {
            long long ar = s_abase + aex;
            for (int st = 0; st < steps; ++st) {
                const int m = dl + st;
                if (!s_keep[m]) continue;
                const int slot = s_src[m];
                const int rep = MULTI ? (int)skey_rep(s_sk[slot], w.rb) : 0;
                w.att_off[s_base + s_dst[m]] = ar;
                ar += attempts_of(s_val[slot], w.rep[rep].bits, w.dm == 1 ? 2 : 1, c);
            }
        }
        const long long obase = s_base;
        if (obase + tot > w.main_cap) {
            if (threadIdx.x == 0) atomicOr(&c->err, ERR_MAIN_CAP);
        } else {
            for (int m = threadIdx.x; m < la + lb; m += MG_T) {
                if (!s_keep[m]) continue;
                const long long o = obase + s_dst[m];
                const int slot = s_src[m];
                const uint64_t sk = s_sk[slot];
                const int rep = MULTI ? (int)skey_rep(sk, w.rb) : 0;
                const RepParams &rp = w.rep[rep];
                const DevSys &sy = w.sys[rp.sys];
                const int32_t p = (int32_t)s_val[slot];
                const int32_t ds = s_meta[slot];
                if (stored_skey(MULTI, W)) w.nxt.skey[o] = sk;
                uint64_t key[W];
#pragma unroll
                for (int x = 0; x < W; ++x) {
                    key[x] = s_key[x][slot];
                    w.nxt.key[(size_t)x * w.main_cap + o] = key[x];
                }
                w.nxt.pop[o] = p;
                w.nxt.kdiag[o] = s_kd[slot];
                w.newdet[o] = slot >= la ? 1 : 0;
                if (ss) w.nxt.dslot[o] = ds;
                if (ds >= 0) w.ds.pos[(size_t)rep * w.ds.n + ds] = (int32_t)o;
                const long long ap = p < 0 ? -(long long)p : (long long)p;
                acc_switch(acc, rep, tab, rl, w.acc);
                any = true;
                acc.v[F_NW] += ap;
                acc.v[F_NOCC] += 1;
                if constexpr (is_pair(KIND)) {
                    // density matrix (Sec. 2.3): the trace sum_i rho_ii and
                    // Tr(rho H) = sum rho_ij H_ji over pairs at most doubly excited
                    constexpr int BK = base_kind(KIND), WH = W / 2;
                    uint64_t a[WH], b[WH];
                    int nd = 0;
#pragma unroll
                    for (int x = 0; x < WH; ++x) {
                        a[x] = key[x];
                        b[x] = key[WH + x];
                        nd += __popcll(a[x] ^ b[x]);
                    }
                    if (nd == 0) {
                        acc.v[F_N0] += p;
                        add_limbs(acc.v, diag_element<BK, WH>(sy, a) * (double)p);
                    } else if (nd == 2 || nd == 4) {
                        add_limbs(acc.v, hij<BK, WH>(sy, b, a) * (double)p);
                    }
                } else {
                    const uint64_t(&ref)[W] = *(const uint64_t(*)[W])sy.ref;
                    int nd = 0;
#pragma unroll
                    for (int x = 0; x < W; ++x) nd += __popcll(key[x] ^ ref[x]);
                    if (nd == 0) {
                        acc.v[F_N0] += p;
                    } else if (nd == 2 || nd == 4) {
                        const double hv = hij<KIND, W>(sy, ref, key);
                        add_limbs(acc.v, hv * (double)p);
                    }
                }
            }
        }
        if (tile == ntiles - 1 && threadIdx.x == 0) {
            c->n_main_new = obase + tot;
            if (obase + tot <= w.main_cap) w.att_off[obase + tot] = s_abase + atot;
            c->n_att_new = s_abase + atot;
        }
        __syncthreads();
    }
    acc_finish(acc, any && acc.rep >= 0, tab, rl, w.acc, w.part_mrg);
    if (ts) ts_finish<true>(w, kd_max, kd_rep, kd_max > -INFINITY);
    if (blockIdx.x == 0 && threadIdx.x == 0 && ntiles == 0) {
        c->n_main_new = 0;
        w.att_off[0] = 0;
        c->n_att_new = 0;
    }
}

// The diagonal element death uses, relative to H_00: K_ii for a determinant;
// for a pair (i, j) of the density-matrix methods (Sec. 2.3) (K_ii + K_jj) / 2
// (DMQMC, the symmetrised Bloch equation) or K_jj - K_ii (IP-DMQMC, with H^0
// the diagonal part of H).
template <int KIND, int W>
__device__ double entry_kdiag(const Work &w, const DevSys &sy, const uint64_t (&key)[W])
{
    if constexpr (is_pair(KIND)) {
        constexpr int BK = base_kind(KIND), WH = W / 2;
        uint64_t a[WH], b[WH];
#pragma unroll
        for (int x = 0; x < WH; ++x) {
            a[x] = key[x];
            b[x] = key[WH + x];
        }
        const double ki = diag_element<BK, WH>(sy, a) - sy.H00;
        const double kj = diag_element<BK, WH>(sy, b) - sy.H00;
        return w.dm == 1 ? (ki + kj) * 0.5 : kj - ki;
    } else {
        return diag_element<KIND, W>(sy, key) - sy.H00;
    }
}

// K_jj - H_00 of the determinants the merge has just created (marked NaN).
// Each block scans a chunk of the new list, queues the marked entries in LDS
// and evaluates them one per thread, so no lane idles on unmarked entries;
// for a single replica the diagonal's tables are read from LDS.
// Chunks of 16384 flags: new determinants are a few per cent of the list, and
// a chunk must hold enough of them to fill the block's waves (at 4096 flags a
// 256-thread block had about one partial wave of work per chunk)
constexpr int ND_T = 512, ND_CHUNK = 16384;
static_assert(ND_CHUNK == ND_T * 32, "each thread scans 32 new-determinant flags");

template <int KIND, int W>
__global__ __launch_bounds__(ND_T) void k_new_diag(Work w)
{
    const Ctl *c = w.ctl;
    if (c->err) return;
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    __shared__ uint16_t s_q[ND_CHUNK];  // offsets of the chunk's new determinants
    __shared__ int s_n;
    const long long n = c->n_main_new;
    const DevSys &s0 = w.sys[w.rep[0].sys];
    // the host stages tables only when every replica has the same system
    const bool local = w.lds_diag > 0 && (KIND == K_UEG || KIND == K_MOLECULAR);
    UegTables lu = s0.u;
    const double *lhd = s0.hd, *lJ = s0.Jt, *lK = s0.Kt;
    if (local) {
        double *t0 = (double *)dyn_lds;
        const int m = s0.n_spatial;
        if (KIND == K_UEG) {
            if (8 * (m + m * m) <= ND_LDS_MAX) {
                // kinetic energies and the exchange table v(|n_p - n_q|^2)
                double *t1 = t0 + m;
                for (int i = threadIdx.x; i < m; i += ND_T) t0[i] = lu.eps[i];
                for (int i = threadIdx.x; i < m * m; i += ND_T) t1[i] = lu.vx[i];
                lu.eps = t0;
                lu.vx = t1;
            } else {
                // large bases: kinetic energies, v by |dn|^2 and the packed momenta
                const int nv = s0.vlen;
                double *t1 = t0 + m;
                int32_t *t2 = (int32_t *)(t1 + nv);
                for (int i = threadIdx.x; i < m; i += ND_T) t0[i] = lu.eps[i];
                for (int i = threadIdx.x; i < nv; i += ND_T) t1[i] = lu.vtab[i];
                for (int i = threadIdx.x; i < m; i += ND_T) t2[i] = lu.npk[i];
                lu.eps = t0;
                lu.vtab = t1;
                lu.npk = t2;
                lu.vx = nullptr;
            }
        } else {
            double *t1 = t0 + m, *t2 = t1 + m * m;
            for (int i = threadIdx.x; i < m; i += ND_T) t0[i] = lhd[i];
            for (int i = threadIdx.x; i < m * m; i += ND_T) {
                t1[i] = lJ[i];
                t2[i] = lK[i];
            }
            lhd = t0;
            lJ = t1;
            lK = t2;
        }
    }
    for (long long base = (long long)blockIdx.x * ND_CHUNK; base < n; base += (long long)gridDim.x * ND_CHUNK) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        // the merge's new-determinant flags, 32 per thread in two 16-byte loads
        {
            const int q0 = threadIdx.x * 32;
            const long long i0 = base + q0;
            if (i0 + 32 <= n) {
                const uint4 f0 = *(const uint4 *)(w.newdet + i0);
                const uint4 f1 = *(const uint4 *)(w.newdet + i0 + 16);
                const uint32_t fw[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
                for (int b = 0; b < 32; ++b)
                    if ((fw[b >> 2] >> (8 * (b & 3))) & 0xFFu) s_q[atomicAdd(&s_n, 1)] = (uint16_t)(q0 + b);
            } else {
                for (int b = 0; b < 32 && i0 + b < n; ++b)
                    if (w.newdet[i0 + b]) s_q[atomicAdd(&s_n, 1)] = (uint16_t)(q0 + b);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < s_n; q += ND_T) {
            const long long i = base + s_q[q];
            uint64_t key[W];
#pragma unroll
            for (int x = 0; x < W; ++x) key[x] = w.nxt.key[(size_t)x * w.main_cap + i];
            if (local) {
                double e;
                if constexpr (KIND == K_UEG) {
                    e = diag_ueg<W>(lu, key);
                } else {
                    const int m = s0.n_spatial;
                    e = 0.0;
                    for_bits<W>(key, [&](int P) { e = e + lhd[P >> 1]; });
                    for_pairs<W>(key, [&](int P, int Q) {
                        const int p = P >> 1, q = Q >> 1;
                        const double x = lJ[p * m + q];
                        const double y = ((P & 1) == (Q & 1)) ? lK[p * m + q] : 0.0;
                        e = e + (x - y);
                    });
                }
                w.nxt.kdiag[i] = e - s0.H00;
            } else {
                const int rep = w.rb ? (int)skey_rep(w.nxt.skey[i], w.rb) : 0;
                const DevSys &sy = w.sys[w.rep[rep].sys];
                w.nxt.kdiag[i] = entry_kdiag<KIND, W>(w, sy, key);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// deterministic projection (Sec. 2.1 semi-stochastic): y = K_DD n_D, summed
// exactly in fixed point and rounded once (FP64 mode), or as BF16 x3 products
// with FP32 accumulation (split mode); then n_D += SR(-dtau (y - S n_D))
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void k_det_gather(Work w)
{
    const Ctl *c = w.ctl;
    if (c->err || !c->ss_active) return;
    const int n = w.ds.n, np = w.ds.npad;
    const int nd = n * w.R;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x)
        w.ds.c[i] = (double)w.cur.pop[w.ds.pos[i]];
    if (w.ds.precision == 1) {
        // BF16 hi/lo split of the amplitudes (zero padded to npad)
        const int tot = np * w.R;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
            const int r = i / np, j = i % np;
            const float cf = j < n ? (float)w.cur.pop[w.ds.pos[r * n + j]] : 0.0f;
            const uint16_t hi = bf16_rn(cf);
            w.ds.Chi[i] = hi;
            w.ds.Clo[i] = bf16_rn(cf - bf16_f(hi));
        }
    }
}

// rounded increment of a deterministic entry: n += SR(-dtau (y - S n))
__device__ __forceinline__ void det_update(const Work &w, const Ctl *c, int rep, long long row, double y, double nv)
{
    const RepParams &rp = w.rep[rep];
    const double delta = (-rp.tau) * (y - w.shift[rep] * nv);
    const U4 r = draw(TAG_SEMISTOCH, 0, c->t, w.ds.h64[row], rp.k0, rp.k1);
    const double u = u53(r.x, r.y);
    if (!(fabs(delta) < 0x1p40)) atomicOr(&((Ctl *)c)->err, ERR_OVERFLOW);
    const long long k = delta >= 0.0 ? sround(delta, u) : -sround(-delta, u);
    w.ds.y[row] = y;
    w.ds.delta[row] = k;
}

// mode 0: the FP64 projection of the iteration. mode 1 (split precision, every
// check_period iterations): FP64 reference y and the error of the split result
// relative to sum_j |K_ij||c_j|, maximised into the replica's estimators.
__global__ __launch_bounds__(256) void k_det_project_fp64(Work w, int mode)
{
    const Ctl *c = w.ctl;
    if (c->err || !c->ss_active) return;
    if (mode == 1 && (w.ds.precision != 1 || w.ds.check_period <= 0 || c->t % (uint32_t)w.ds.check_period != 0))
        return;
    const int n = w.ds.n;
    const int lane = lane_id();
    const long long rows = (long long)n * w.R;
    for (long long job = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); job < rows;
         job += (long long)gridDim.x * (blockDim.x >> 6)) {
        // shared space: the replicas of one row of K_DD are consecutive jobs
        // (the row is read once from memory)
        const int rep = w.ds.shared ? (int)(job % w.R) : (int)(job / n);
        const int d = w.ds.shared ? (int)(job / w.R) : (int)(job % n);
        const long long row = (long long)rep * n + d;
        const double *K = w.ds.K + ((size_t)(w.ds.shared ? 0 : rep) * n + d) * n;
        const double *cv = w.ds.c + (size_t)rep * n;
        // y = sum_j K_ij n_j, exact in fixed point (2^-64), rounded once: the
        // order of the terms over lanes and the wave reduction does not matter
        long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        double pabs = 0.0;
        for (int j = lane; j < n; j += 64) {
            add_limbs4(a0, a1, a2, a3, K[j] * cv[j]);
            if (mode == 1) pabs = pabs + fabs(K[j]) * fabs(cv[j]);
        }
        a0 = wave_sum<long long>(a0);
        a1 = wave_sum<long long>(a1);
        a2 = wave_sum<long long>(a2);
        a3 = wave_sum<long long>(a3);
        if (mode == 1) pabs = wave_sum<double>(pabs);
        if (lane == 0) {
            const double part = limbs_to_double(a0, a1, a2, a3);
            if (mode == 0) {
                det_update(w, c, rep, row, part, cv[d]);
            } else {
                w.ds.yref[row] = part;
                const double e = pabs > 0.0 ? fabs(w.ds.y[row] - part) / pabs : 0.0;
                atomicMax((unsigned long long *)&w.acc[rep].ss_err, (unsigned long long)__double_as_longlong(e));
            }
        }
    }
}

// Split-precision projection on MFMA: y = K c with K and c split into BF16
// hi + lo planes, y = K_hi c_hi + K_hi c_lo + K_lo c_hi accumulated in FP32
// (the "bf16x3" scheme) with v_mfma_f32_16x16x32_bf16. A block computes 16
// rows of up to 16 replicas (one K_DD shared by all) or of one replica (its
// amplitudes in column 0 of the 16 x 16 B tile).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int DP_WAVES = 8;  // waves per block of the split projection (split over k)

__global__ __launch_bounds__(64 * DP_WAVES) void k_det_project_split(Work w)
{
    // One block per job (16 rows x up to 16 columns of Y = K C); its waves
    // take interleaved 32-wide steps of the k range (gfx950's 16x16x32 BF16
    // MFMA: each lane holds 8 consecutive k of its row of A and of its column
    // of B, loaded with the same k order so the dot products pair correctly)
    // and their FP32 partial tiles are summed in LDS in wave order. Shared
    // space: the columns are 16 replicas, one K_DD for all. Otherwise: one
    // replica per job, in column 0.
    const Ctl *c = w.ctl;
    if (c->err || !c->ss_active || w.ds.precision != 1) return;
    __shared__ float s_part[DP_WAVES][64][4];
    const int n = w.ds.n, np = w.ds.npad;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int tiles = np / 16;
    const bool shared = w.ds.shared != 0;
    const int cblocks = shared ? (w.R + 15) / 16 : w.R;
    const long long jobs = (long long)tiles * cblocks;
    for (long long job = blockIdx.x; job < jobs; job += gridDim.x) {
        const int rt = (int)(job / cblocks), cb = (int)(job % cblocks);
        const int arow = rt * 16 + (lane & 15);
        const int kq = 8 * (lane >> 4);
        // this lane's column of B (and of the result): a replica
        const int rep = shared ? cb * 16 + (lane & 15) : cb;
        const bool bval = shared ? rep < w.R : (lane & 15) == 0;
        const size_t kmat = shared ? 0 : (size_t)cb;
        const uint16_t *kh = w.ds.Khi + (kmat * np + arow) * np + kq;
        const uint16_t *kl = w.ds.Klo + (kmat * np + arow) * np + kq;
        const uint16_t *ch = w.ds.Chi + (size_t)(bval ? rep : 0) * np + kq;
        const uint16_t *cl = w.ds.Clo + (size_t)(bval ? rep : 0) * np + kq;
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
        const bf16x8_t zero = {};
        for (int kk = 32 * wv; kk < np; kk += 32 * DP_WAVES) {
            const bf16x8_t ah = *(const bf16x8_t *)(kh + kk);
            const bf16x8_t al = *(const bf16x8_t *)(kl + kk);
            bf16x8_t bh = zero, bl = zero;
            if (bval) {
                bh = *(const bf16x8_t *)(ch + kk);
                bl = *(const bf16x8_t *)(cl + kk);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) s_part[wv][lane][i] = acc[i];
        __syncthreads();
        // lane holds rows 4 (lane / 16) + i of column lane % 16
        if (wv == 0 && bval) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float y = s_part[0][lane][i];
                for (int q = 1; q < DP_WAVES; ++q) y = y + s_part[q][lane][i];
                const int d = rt * 16 + 4 * (lane >> 4) + i;
                if (d < n) {
                    const long long row = (long long)rep * n + d;
                    det_update(w, c, rep, row, (double)y, w.ds.c[row]);
                }
            }
        }
        __syncthreads();
    }
}

// BF16 hi/lo planes of K_DD (zero padded to npad), once per deterministic space
__global__ void k_split_planes(Work w)
{
    const int n = w.ds.n, np = w.ds.npad;
    const long long tot = (long long)w.ds.nk * np * np;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(x / ((long long)np * np));
        const int i = (int)((x / np) % np), j = (int)(x % np);
        float k = 0.0f;
        if (i < n && j < n) k = (float)w.ds.K[((size_t)r * n + i) * n + j];
        const uint16_t hi = bf16_rn(k);
        w.ds.Khi[x] = hi;
        w.ds.Klo[x] = bf16_rn(k - bf16_f(hi));
    }
}

// explicit instantiations
#define FQ_INSTM(KIND, W, MI)                                    \
    template __global__ void k_merge<KIND, W, false, MI>(Work);   \
    template __global__ void k_merge<KIND, W, true, MI>(Work);
#define FQ_INSTS(KIND, W, SI)                                            \
    template __global__ void k_spawn<KIND, W, false, false, SI>(Work);    \
    template __global__ void k_spawn<KIND, W, true, false, SI>(Work);
#define FQ_INSTT(KIND, W, SI)                                            \
    template __global__ void k_spawn<KIND, W, false, true, SI>(Work);     \
    template __global__ void k_spawn<KIND, W, true, true, SI>(Work);
#define FQ_INST(KIND, W)                                          \
    template __global__ void k_new_diag<KIND, W>(Work);            \
    FQ_INSTM(KIND, W, 2)
// keys of up to two words: the 1- and 4-position merge tiles as well
#define FQ_INST_SHORT(KIND, W) \
    FQ_INST(KIND, W)           \
    FQ_INSTM(KIND, W, 1)       \
    FQ_INSTM(KIND, W, 4)
// spawn kernels of one kind and key width over the attempts-per-thread variants
#define FQ_SPAWN3(KIND, W) FQ_INSTS(KIND, W, 2) FQ_INSTS(KIND, W, 4) FQ_INSTS(KIND, W, 8)
#define FQ_SPAWN3T(KIND, W) FQ_INSTT(KIND, W, 2) FQ_INSTT(KIND, W, 4) FQ_INSTT(KIND, W, 8)
FQ_INST_SHORT(K_HUBBARD, 1)
FQ_INST_SHORT(K_UEG, 1)
FQ_INST_SHORT(K_UEG, 2)
FQ_INST(K_UEG, 4)
FQ_INST(K_UEG, 8)
FQ_INST_SHORT(K_MOLECULAR, 1)
FQ_INST_SHORT(K_MOLECULAR, 2)
// pairs of one-word determinants (density-matrix methods)
FQ_INST_SHORT(K_HUBBARD | K_PAIR, 2)
FQ_INST_SHORT(K_UEG | K_PAIR, 2)
FQ_INST_SHORT(K_MOLECULAR | K_PAIR, 2)
FQ_SPAWN3(K_HUBBARD, 1)
FQ_SPAWN3(K_UEG, 1)
FQ_SPAWN3(K_UEG, 2)
FQ_SPAWN3(K_MOLECULAR, 1)
FQ_SPAWN3(K_MOLECULAR, 2)
FQ_SPAWN3T(K_UEG, 1)
FQ_SPAWN3T(K_UEG, 2)
FQ_SPAWN3T(K_MOLECULAR, 1)
FQ_SPAWN3T(K_MOLECULAR, 2)
FQ_INSTS(K_UEG, 4, 2)
FQ_INSTS(K_UEG, 8, 2)
FQ_INSTT(K_UEG, 4, 2)
FQ_INSTT(K_UEG, 8, 2)
FQ_INSTS(K_HUBBARD | K_PAIR, 2, 4)
FQ_INSTS(K_UEG | K_PAIR, 2, 4)
FQ_INSTS(K_MOLECULAR | K_PAIR, 2, 4)
#define FQ_INSTW(W)                                        \
    template __global__ void k_reduce<W>(Work, int);       \
    template __global__ void k_fixup<W>(Work);             \
    template __global__ void k_merge_partition<W, 2>(Work);
FQ_INSTW(1)
FQ_INSTW(2)
FQ_INSTW(4)
FQ_INSTW(8)
template __global__ void k_merge_partition<1, 1>(Work);
template __global__ void k_merge_partition<1, 4>(Work);
template __global__ void k_merge_partition<2, 1>(Work);
template __global__ void k_merge_partition<2, 4>(Work);
template __global__ void k_sort_pass<8>(Work, int, const uint64_t *, const uint32_t *, uint64_t *, uint32_t *);
template __global__ void k_sort_pass<12>(Work, int, const uint64_t *, const uint32_t *, uint64_t *, uint32_t *);
template __global__ void k_sort_pass<16>(Work, int, const uint64_t *, const uint32_t *, uint64_t *, uint32_t *);

}  // namespace fq

// ---------------------------------------------------------------------------
// set-up kernels: H_00 per system, K_ii - H_00 and attempt counts of a list,
// K_DD of a deterministic space
// ---------------------------------------------------------------------------
namespace fq {

template <int KIND, int W>
__global__ void k_h00(DevSys *sys, int n_sys)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_sys) return;
    uint64_t ref[W];
#pragma unroll
    for (int q = 0; q < W; ++q) ref[q] = sys[i].ref[q];
    sys[i].H00 = diag_element<KIND, W>(sys[i], ref);
}

template <int KIND, int W>
__global__ void k_kdiag(Work w, MainList L, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        uint64_t key[W];
#pragma unroll
        for (int q = 0; q < W; ++q) key[q] = L.key[(size_t)q * w.main_cap + i];
        const int rep = (int)skey_rep(L.skey[i], w.rb);
        const RepParams rp = w.rep[rep];
        const DevSys &sy = w.sys[rp.sys];
        L.kdiag[i] = entry_kdiag<KIND, W>(w, sy, key);
        const int32_t p = L.pop[i];
        const long long ap = p < 0 ? -(long long)p : (long long)p;
        L.natt[i] = (int32_t)((w.dm == 1 ? 2 : 1) * (rp.bits == 0 ? ap : ((ap + (1ll << rp.bits) - 1) >> rp.bits)));
    }
}

// K[rep][d][e] = <D_d|H|D_e> - H_00 delta_de for D keys given in D order
template <int KIND, int W>
__global__ void k_build_kdd(Work w, const uint64_t *dkeys /* [W][R*n] */, double *K)
{
    const int n = w.ds.n;
    const int nd = n * w.R;
    const long long tot = (long long)w.ds.nk * n * n;  // shared space: replica 0's keys (the same for all)
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += (long long)gridDim.x * blockDim.x) {
        const int rep = (int)(x / ((long long)n * n));
        const int d = (int)((x / n) % n), e = (int)(x % n);
        uint64_t a[W], b[W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            a[q] = dkeys[(size_t)q * nd + (size_t)rep * n + d];
            b[q] = dkeys[(size_t)q * nd + (size_t)rep * n + e];
        }
        const DevSys &sy = w.sys[w.rep[rep].sys];
        double v;
        if (d == e)
            v = diag_element<KIND, W>(sy, a) - sy.H00;
        else
            v = hij<KIND, W>(sy, a, b);
        K[x] = v;
    }
}

#define FQ_INST2(KIND, W)                                                     \
    template __global__ void k_h00<KIND, W>(DevSys *, int);                 \
    template __global__ void k_kdiag<KIND, W>(Work, MainList, long long);   \
    template __global__ void k_build_kdd<KIND, W>(Work, const uint64_t *, double *);
FQ_INST2(K_HUBBARD, 1)
FQ_INST2(K_UEG, 1)
FQ_INST2(K_UEG, 2)
FQ_INST2(K_UEG, 4)
FQ_INST2(K_UEG, 8)
FQ_INST2(K_MOLECULAR, 1)
FQ_INST2(K_MOLECULAR, 2)
template __global__ void k_kdiag<K_HUBBARD | K_PAIR, 2>(Work, MainList, long long);
template __global__ void k_kdiag<K_UEG | K_PAIR, 2>(Work, MainList, long long);
template __global__ void k_kdiag<K_MOLECULAR | K_PAIR, 2>(Work, MainList, long long);

// ---------------------------------------------------------------------------
// launchers used by the host library
// ---------------------------------------------------------------------------
// spawning, SI attempts per thread: LDS-staged generator tables when the
// host staged them, the multi-replica kernel for several instances
template <int KIND, int W, int SI>
static void launch_spawn(const Work &w, const Grids &g, hipStream_t s)
{
    constexpr bool TAB = KIND == K_UEG || KIND == K_MOLECULAR;
    if (w.R > 1 && TAB && w.lds_tables > 0)
        k_spawn<KIND, W, true, TAB, SI><<<g.spawn, SP_T, g.spawn_lds, s>>>(w);
    else if (w.R > 1)
        k_spawn<KIND, W, true, false, SI><<<g.spawn, SP_T, 0, s>>>(w);
    else if (TAB && w.lds_tables > 0)
        k_spawn<KIND, W, false, TAB, SI><<<g.spawn, SP_T, g.spawn_lds, s>>>(w);
    else
        k_spawn<KIND, W, false, false, SI><<<g.spawn, SP_T, 0, s>>>(w);
}

// merge partition and merge, MI positions per thread (rec: records the event
// after each launch)
template <int KIND, int W, int MI, typename Rec>
static void launch_merge(const Work &w, const Grids &g, hipStream_t s, int accb, Rec &rec)
{
    k_merge_partition<W, MI><<<g.part, 256, 0, s>>>(w);
    rec();
    if (w.R > 1)
        k_merge<KIND, W, true, MI><<<g.merge, MergeCfg<W, MI>::T, accb, s>>>(w);
    else
        k_merge<KIND, W, false, MI><<<g.merge, MergeCfg<W, MI>::T, accb, s>>>(w);
    rec();
}

template <int KIND, int W>
static void launch_kind(const Work &w, const Grids &g, hipStream_t s, hipEvent_t *ev)
{
    // ev (optional): N_KERNEL_SLOTS + 1 events, one before the first launch and
    // one after every launch of the iteration
    int e = 0;
    auto rec = [&]() {
        if (ev) (void)hipEventRecord(ev[e++], s);
    };
    rec();
    k_begin<<<1, 256, 0, s>>>(w);
    rec();
    // attempts per thread: a tile-shape variant for keys of up to two words
    constexpr bool VAR = W <= 2 && !is_pair(KIND);
    int si = VAR ? g.spawn_i : (W <= 2 ? 4 : 2);
    if (si != 2 && si != 8) si = W <= 2 ? 4 : 2;  // the partition must match the launched variant
    k_spawn_partition<<<g.part, 256, 0, s>>>(w, SP_T * si);
    rec();
    if (si == 2)
        launch_spawn<KIND, W, VAR ? 2 : (W <= 2 ? 4 : 2)>(w, g, s);
    else if (si == 8)
        launch_spawn<KIND, W, VAR ? 8 : (W <= 2 ? 4 : 2)>(w, g, s);
    else
        launch_spawn<KIND, W, W <= 2 ? 4 : 2>(w, g, s);
    rec();
    if (w.ccmc_trunc > 0) (void)enqueue_ccmc(0, KIND, w, g, s);
    rec();
    k_sort_hist<<<g.hist, 256, 0, s>>>(w);
    rec();
    uint64_t *K[2] = {w.sp.skey, w.sp.skey2};
    uint32_t *I[2] = {w.sp.idx, w.sp.idx2};
    for (int p = 0; p < 8; ++p) {
        const uint64_t *ki = K[p & 1];
        const uint32_t *ii = p == 0 ? nullptr : I[p & 1];
        if (g.sort_i == 8)
            k_sort_pass<8><<<g.sort, OS_T, 0, s>>>(w, p, ki, ii, K[(p + 1) & 1], I[(p + 1) & 1]);
        else if (g.sort_i == 16)
            k_sort_pass<16><<<g.sort, OS_T, 0, s>>>(w, p, ki, ii, K[(p + 1) & 1], I[(p + 1) & 1]);
        else
            k_sort_pass<12><<<g.sort, OS_T, 0, s>>>(w, p, ki, ii, K[(p + 1) & 1], I[(p + 1) & 1]);
        rec();
    }
    const int accb = acc_rows(w.R) * EST_FIELDS * 8;
    k_reduce<W><<<g.reduce, RD_T, accb, s>>>(w, 0);
    rec();
    k_fixup<W><<<g.fixup, 256, 0, s>>>(w);
    rec();
    k_reduce<W><<<g.reduce, RD_T, accb, s>>>(w, 1);
    rec();
    k_det_gather<<<g.det, 256, 0, s>>>(w);
    rec();
    if (w.ds.precision == 1)
        k_det_project_split<<<g.det, 64 * DP_WAVES, 0, s>>>(w);
    else
        k_det_project_fp64<<<g.det, 256, 0, s>>>(w, 0);
    rec();
    k_det_project_fp64<<<g.det, 256, 0, s>>>(w, 1);
    rec();
    const int mi = W <= 2 ? g.merge_i : 2;
    if (mi == 1) {
        launch_merge<KIND, W, W <= 2 ? 1 : 2>(w, g, s, accb, rec);
    } else if (mi == 4) {
        launch_merge<KIND, W, W <= 2 ? 4 : 2>(w, g, s, accb, rec);
    } else {
        launch_merge<KIND, W, 2>(w, g, s, accb, rec);
    }
    k_new_diag<KIND, W><<<g.newdiag, ND_T, w.lds_diag, s>>>(w);
    rec();
    if (w.ccmc_trunc > 0) (void)enqueue_ccmc(1, KIND, w, g, s);
    rec();
    k_end<<<w.R, 1024, 0, s>>>(w, g.reduce, g.merge);
    rec();
}

hipError_t enqueue_iteration(const Work &w, int kind, const Grids &g, hipStream_t s, hipEvent_t *ev)
{
    switch (kind * 16 + w.W) {
    case K_HUBBARD * 16 + 1: launch_kind<K_HUBBARD, 1>(w, g, s, ev); break;
    case K_UEG * 16 + 1: launch_kind<K_UEG, 1>(w, g, s, ev); break;
    case K_UEG * 16 + 2: launch_kind<K_UEG, 2>(w, g, s, ev); break;
    case K_UEG * 16 + 4: launch_kind<K_UEG, 4>(w, g, s, ev); break;
    case K_UEG * 16 + 8: launch_kind<K_UEG, 8>(w, g, s, ev); break;
    case K_MOLECULAR * 16 + 1: launch_kind<K_MOLECULAR, 1>(w, g, s, ev); break;
    case K_MOLECULAR * 16 + 2: launch_kind<K_MOLECULAR, 2>(w, g, s, ev); break;
    case (K_HUBBARD | K_PAIR) * 16 + 2: launch_kind<K_HUBBARD | K_PAIR, 2>(w, g, s, ev); break;
    case (K_UEG | K_PAIR) * 16 + 2: launch_kind<K_UEG | K_PAIR, 2>(w, g, s, ev); break;
    case (K_MOLECULAR | K_PAIR) * 16 + 2: launch_kind<K_MOLECULAR | K_PAIR, 2>(w, g, s, ev); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, int W>
static void setup_kind(int what, const Work &w, DevSys *sys, int n_sys, MainList L, long long n, const uint64_t *dk,
                       double *K, hipStream_t s)
{
    // H_00 of the reference determinant (for pairs: of one half)
    if (what == 0) k_h00<base_kind(KIND), is_pair(KIND) ? W / 2 : W><<<(n_sys + 63) / 64, 64, 0, s>>>(sys, n_sys);
    if (what == 1) {
        if (n > 0) k_kdiag<KIND, W><<<(int)std::min<long long>((n + 255) / 256, 4096), 256, 0, s>>>(w, L, n);
        Work w2 = w;
        w2.cur = L;
        k_scan_attempts<<<256, SCAN_T, 0, s>>>(w2);
    }
    if constexpr (!is_pair(KIND)) {
        if (what == 2) {
            k_build_kdd<KIND, W><<<2048, 256, 0, s>>>(w, dk, K);
            if (w.ds.precision == 1) k_split_planes<<<2048, 256, 0, s>>>(w);
        }
    }
}

hipError_t enqueue_setup(int what, int kind, const Work &w, DevSys *sys, int n_sys, MainList L, long long n,
                         const uint64_t *dk, double *K, hipStream_t s)
{
    switch (kind * 16 + w.W) {
    case K_HUBBARD * 16 + 1: setup_kind<K_HUBBARD, 1>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_UEG * 16 + 1: setup_kind<K_UEG, 1>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_UEG * 16 + 2: setup_kind<K_UEG, 2>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_UEG * 16 + 4: setup_kind<K_UEG, 4>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_UEG * 16 + 8: setup_kind<K_UEG, 8>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_MOLECULAR * 16 + 1: setup_kind<K_MOLECULAR, 1>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case K_MOLECULAR * 16 + 2: setup_kind<K_MOLECULAR, 2>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case (K_HUBBARD | K_PAIR) * 16 + 2: setup_kind<K_HUBBARD | K_PAIR, 2>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case (K_UEG | K_PAIR) * 16 + 2: setup_kind<K_UEG | K_PAIR, 2>(what, w, sys, n_sys, L, n, dk, K, s); break;
    case (K_MOLECULAR | K_PAIR) * 16 + 2:
        setup_kind<K_MOLECULAR | K_PAIR, 2>(what, w, sys, n_sys, L, n, dk, K, s);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int occupancy_blocks(int which)
{
    int nb = 1;
    hipError_t e = hipSuccess;
    switch (which) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sort_pass<12>, OS_T, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_merge<K_UEG, 2, false, 2>, MergeCfg<2, 2>::T, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_merge<K_UEG, 8, false, 2>, MergeCfg<8, 2>::T, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_reduce<2>, RD_T, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_scan_attempts, SCAN_T, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_spawn<K_UEG, 2, false, true, 4>, SP_T, 8192); break;
    default: break;
    }
    if (e != hipSuccess) nb = 1;  // a persistent grid of one block per CU still covers every tile
    return nb < 1 ? 1 : nb;
}

}  // namespace fq
