// Device-side building blocks of the FCIQMC iteration for gfx950: counter
// based random numbers, determinant hashing, bit-string algebra, the three
// systems' Slater-Condon matrix elements and excitation generators.
//
// Every floating-point expression is written in the order the method defines
// it and compiled with contraction off, so products and sums round exactly as
// written (IEEE double, round to nearest). Only +, -, *, /, floor and fabs are
// used on the per-walker path; transcendental constants arrive precomputed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fq {

constexpr int MAXW = 8;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies with a Weyl key schedule. Counter = (tag << 28 | attempt,
// iteration, hash_lo, hash_hi), key = (seed_lo, seed_hi ^ replica): every draw
// is a pure function of what it is used for, independent of list order.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    return U4{c0, c1, c2, c3};
}

enum : uint32_t { TAG_SELECT = 0, TAG_SELECT2 = 1, TAG_SPAWN_ROUND = 2, TAG_DEATH = 3, TAG_SEMISTOCH = 4, TAG_CLUSTER = 5 };

__device__ __forceinline__ U4 draw(uint32_t tag, uint32_t attempt, uint32_t t, uint64_t h, uint32_t k0,
                                   uint32_t k1)
{
    return philox((tag << 28) | attempt, t, (uint32_t)h, (uint32_t)(h >> 32), k0, k1);
}

// uniform double in [0, 1) with 53 random bits: 32 from a, 21 from b
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * 0x1p-53;
}

// integer in [0, n): floor(w n / 2^32)
__device__ __forceinline__ uint32_t pick(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

// stochastic rounding of m >= 0: floor(m) + [u < m - floor(m)]
__device__ __forceinline__ int64_t sround(double m, double u)
{
    const double f = floor(m);
    int64_t k = (int64_t)f;
    if (u < m - f) k += 1;
    return k;
}

// ---------------------------------------------------------------------------
// Determinant hash: MurmurHash64A (Appleby; the paper's code hashes with
// MurmurHash2) over the 8W bytes of the key. For W = 1 every step is a
// bijection of the word, so distinct one-word keys never collide.
// ---------------------------------------------------------------------------
constexpr uint64_t HASH_SEED = 0x9E3779B97F4A7C15ull;

template <int W>
__device__ __forceinline__ uint64_t hash64(const uint64_t (&k)[W])
{
    const uint64_t m = 0xc6a4a7935bd1e995ull;
    uint64_t h = HASH_SEED ^ ((uint64_t)(8 * W) * m);
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint64_t x = k[i];
        x *= m;
        x ^= x >> 47;
        x *= m;
        h ^= x;
        h *= m;
    }
    h ^= h >> 47;
    h *= m;
    h ^= h >> 47;
    return h;
}

// sort key: replica id in the top rb bits, hash below
__device__ __forceinline__ uint64_t make_skey(uint64_t h, uint32_t rep, int rb)
{
    return rb ? (((uint64_t)rep << (64 - rb)) | (h >> rb)) : h;
}
__device__ __forceinline__ uint32_t skey_rep(uint64_t s, int rb) { return rb ? (uint32_t)(s >> (64 - rb)) : 0u; }

// ---------------------------------------------------------------------------
// bit strings
// ---------------------------------------------------------------------------
// Every word is touched with a mask (no array index computed from P): a
// conditional update of one word lets the compiler turn the loop into an
// indexed access, which puts longer keys in scratch memory.
template <int W>
__device__ __forceinline__ int getbit(const uint64_t (&k)[W], int P)
{
    const int wd = P >> 6;
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) x |= (wd == i) ? k[i] : 0ull;
    return (int)((x >> (P & 63)) & 1u);
}
template <int W>
__device__ __forceinline__ void flipbit(uint64_t (&k)[W], int P)
{
    const int wd = P >> 6;
    const uint64_t m = (uint64_t)1 << (P & 63);
#pragma unroll
    for (int i = 0; i < W; ++i) k[i] ^= (wd == i) ? m : 0ull;
}

// mask of bits [lo, hi) within word i
__device__ __forceinline__ uint64_t range_mask(int i, int lo, int hi)
{
    int a = lo - 64 * i, b = hi - 64 * i;
    a = a < 0 ? 0 : (a > 64 ? 64 : a);
    b = b < 0 ? 0 : (b > 64 ? 64 : b);
    if (b <= a) return 0;
    const uint64_t hm = b == 64 ? ~0ull : ((1ull << b) - 1);
    const uint64_t lm = a == 64 ? ~0ull : ((1ull << a) - 1);
    return hm & ~lm;
}

// (-1)^{number of occupied orbitals strictly between P and A}
template <int W>
__device__ __forceinline__ double parity_between(const uint64_t (&k)[W], int P, int A)
{
    const int lo = P < A ? P : A, hi = P < A ? A : P;
    int c = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) c += __popcll(k[i] & range_mask(i, lo + 1, hi));
    return (c & 1) ? -1.0 : 1.0;
}

// position of the r-th (0-based) set bit of a word: choose the 32-bit half,
// then halve the window with 32-bit popcounts
__device__ __forceinline__ int select_in_word(uint64_t x, int r)
{
    const uint32_t lo = (uint32_t)x;
    const int c0 = __popc(lo);
    const bool up = r >= c0;
    uint32_t v = up ? (uint32_t)(x >> 32) : lo;
    int pos = up ? 32 : 0;
    r = up ? r - c0 : r;
#pragma unroll
    for (int s = 16; s > 0; s >>= 1) {
        const int c = __popc(v & ((1u << s) - 1u));
        const bool hi = r >= c;
        r = hi ? r - c : r;
        v = hi ? v >> s : v;
        pos = hi ? pos + s : pos;
    }
    return pos;
}

// position of the r-th set bit of a key, -1 if it has fewer: the word is
// chosen first (selects, no divergence), then searched once
template <int W>
__device__ __forceinline__ int select_bit(const uint64_t (&k)[W], int r)
{
    int wsel = -1;
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const int c = __popcll(k[i]);
        const bool here = wsel < 0 && r < c;
        x = here ? k[i] : x;
        r = (wsel < 0 && !here) ? r - c : r;
        wsel = here ? i : wsel;
    }
    return wsel < 0 ? -1 : 64 * wsel + select_in_word(x, r);
}

template <int W>
__device__ __forceinline__ bool key_eq(const uint64_t (&a)[W], const uint64_t (&b)[W])
{
    bool e = true;
#pragma unroll
    for (int i = 0; i < W; ++i) e = e && (a[i] == b[i]);
    return e;
}

// unsigned big-integer compare: -1, 0, 1
template <int W>
__device__ __forceinline__ int key_cmp(const uint64_t (&a)[W], const uint64_t (&b)[W])
{
    int r = 0;
#pragma unroll
    for (int i = W - 1; i >= 0; --i)
        if (r == 0) r = a[i] < b[i] ? -1 : (a[i] > b[i] ? 1 : 0);
    return r;
}

// ---------------------------------------------------------------------------
// Systems. One DevSys per replica lives in device memory; its tables are
// built on the host from the system description.
// ---------------------------------------------------------------------------
// The UEG tables, as a small view that kernels can point at LDS copies.
struct UegTables {
    const int32_t *npk;   // [M] plane-wave vectors, 10 bits per component biased by 256
    const double *eps;    // kinetic energy per plane wave
    const double *vtab;   // v(|dn|^2)
    const double *vx;     // [M][M] v(|n_p - n_q|^2), or nullptr: use vtab and npk
    const int16_t *grid;  // momentum grid -> plane-wave index, -1 outside
    int32_t M, nel, gmax, gdim;
    // p_gen of an excitation from a same-spin / an opposite-spin pair:
    // 2 / (C(N,2) M) and 2 / (C(N,2) 2M), each one correctly rounded FP64
    // division done on the host (the same value the generator would compute)
    double pgen_same, pgen_opp;
};

struct DevSys {
    int32_t kind, n_spatial, n_so, nel, na, nb;
    int32_t periodic;
    double t, U;
    int32_t vlen, pad0;
    UegTables u;
    const double *h1;     // [n][n]
    const double *eri;    // [n][n][n][n] chemists' notation
    const double *hd;     // [n] h_pp
    const double *Jt;     // [n][n] (pp|qq)
    const double *Kt;     // [n][n] (pq|qp)
    const int64_t *hb_off;  // [n_so][n_so] first entry of pair (P<Q)
    const int32_t *hb_cnt;  // entries of pair
    const double *hb_S;     // [n_so][n_so] total weight of pair
    const uint16_t *hb_AB;  // A | B << 8
    const double *hb_cdf;   // running weight sums
    uint64_t ref[MAXW];
    double H00;
};

enum : int { K_HUBBARD = 1, K_UEG = 2, K_MOLECULAR = 3, K_PAIR = 8 };
// kernels for pairs of determinants (density-matrix methods) take KIND =
// system kind | K_PAIR: a key is the bra's words, then the ket's
__host__ __device__ constexpr bool is_pair(int k) { return (k & K_PAIR) != 0; }
__host__ __device__ constexpr int base_kind(int k) { return k & 7; }

__device__ __forceinline__ double eri_at(const DevSys &s, int p, int q, int r, int t)
{
    const int n = s.n_spatial;
    return s.eri[(((size_t)p * n + q) * n + r) * n + t];
}

// packed plane-wave vectors: component c in bits [10c, 10c + 10), biased by 256;
// sums and differences of a few vectors stay inside each 10-bit field
__device__ __forceinline__ int pk_comp(int32_t v, int c) { return ((v >> (10 * c)) & 1023) - 256; }
__device__ __forceinline__ int pk_dn2(int32_t u, int32_t v)
{
    const int dx = pk_comp(u, 0) - pk_comp(v, 0), dy = pk_comp(u, 1) - pk_comp(v, 1), dz = pk_comp(u, 2) - pk_comp(v, 2);
    return dx * dx + dy * dy + dz * dz;
}

// calls f(P) for every set bit P of a key, in ascending order
template <int W, typename F>
__device__ __forceinline__ void for_bits(const uint64_t (&key)[W], F &&f)
{
#pragma unroll
    for (int wi = 0; wi < W; ++wi) {
        uint64_t m = key[wi];
        while (m) {
            const int P = 64 * wi + __builtin_ctzll(m);
            m &= m - 1;
            f(P);
        }
    }
}

// calls f(P, Q) for every pair P < Q of set bits, P ascending then Q ascending
template <int W, typename F>
__device__ __forceinline__ void for_pairs(const uint64_t (&key)[W], F &&f)
{
    for_bits<W>(key, [&](int P) {
        uint64_t rest[W];
#pragma unroll
        for (int i = 0; i < W; ++i) rest[i] = key[i] & ~range_mask(i, 0, P + 1);
        for_bits<W>(rest, [&](int Q) { f(P, Q); });
    });
}

// UEG: <AB|PQ> - <AB|QP> with momentum conservation
__device__ __forceinline__ double antisym_ueg(const UegTables &u, int A, int B, int P, int Q)
{
    const int sa = A & 1, sb = B & 1, sp = P & 1, sq = Q & 1;
    const int a = A >> 1, b = B >> 1, p = P >> 1, q = Q >> 1;
    const int32_t na = u.npk[a], np = u.npk[p], nq = u.npk[q];
    if (na + u.npk[b] != np + nq) return 0.0;
    double x = 0.0, y = 0.0;
    if (u.vx) {
        if (sa == sp && sb == sq) x = u.vx[p * u.M + a];
        if (sa == sq && sb == sp) y = u.vx[q * u.M + a];
    } else {
        // the same values from v(|dn|^2)
        if (sa == sp && sb == sq) x = u.vtab[pk_dn2(np, na)];
        if (sa == sq && sb == sp) y = u.vtab[pk_dn2(nq, na)];
    }
    return x - y;
}

// UEG diagonal: kinetic energies, then same-spin exchange over pairs P < Q
template <int W>
__device__ double diag_ueg(const UegTables &u, const uint64_t (&key)[W])
{
    double e = 0.0;
    for_bits<W>(key, [&](int P) { e = e + u.eps[P >> 1]; });
    // exchange of the same-spin pairs P < Q, in the order of all pairs (P
    // ascending, then Q ascending): opposite-spin pairs contribute nothing and
    // are not visited
    for_bits<W>(key, [&](int P) {
        const uint64_t sm = (P & 1) ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
        uint64_t rest[W];
#pragma unroll
        for (int i = 0; i < W; ++i) rest[i] = key[i] & sm & ~range_mask(i, 0, P + 1);
        const int p = P >> 1;
        for_bits<W>(rest, [&](int Q) {
            const double v = u.vx ? u.vx[p * u.M + (Q >> 1)] : u.vtab[pk_dn2(u.npk[p], u.npk[Q >> 1])];
            e = e - v;
        });
    });
    return e;
}

// Diagonal element <D|H|D> (Slater-Condon, fixed summation order: one
// ascending sweep of the occupied orbitals, then all pairs P < Q ascending).
template <int KIND, int W>
__device__ double diag_element(const DevSys &s, const uint64_t (&key)[W])
{
    double e = 0.0;
    if constexpr (KIND == K_HUBBARD) {
        const uint64_t k = key[0];
        for (int p = 0; p < s.n_spatial; ++p)
            if (((k >> (2 * p)) & 1) && ((k >> (2 * p + 1)) & 1)) e = e + s.U;
        return e;
    } else if constexpr (KIND == K_UEG) {
        return diag_ueg<W>(s.u, key);
    } else {
        const int n = s.n_spatial;
        for_bits<W>(key, [&](int P) { e = e + s.hd[P >> 1]; });
        for_pairs<W>(key, [&](int P, int Q) {
            const int p = P >> 1, q = Q >> 1;
            const double x = s.Jt[p * n + q];
            const double y = ((P & 1) == (Q & 1)) ? s.Kt[p * n + q] : 0.0;
            e = e + (x - y);
        });
        return e;
    }
}

// <AB|PQ> - <AB|QP> (physicists' notation, spin-orbital indices)
template <int KIND>
__device__ __forceinline__ double antisym(const DevSys &s, int A, int B, int P, int Q)
{
    const int sa = A & 1, sb = B & 1, sp = P & 1, sq = Q & 1;
    const int a = A >> 1, b = B >> 1, p = P >> 1, q = Q >> 1;
    if constexpr (KIND == K_HUBBARD) {
        return 0.0;
    } else if constexpr (KIND == K_UEG) {
        return antisym_ueg(s.u, A, B, P, Q);
    } else {
        const double x = (sa == sp && sb == sq) ? eri_at(s, a, p, b, q) : 0.0;
        const double y = (sa == sq && sb == sp) ? eri_at(s, a, q, b, p) : 0.0;
        return x - y;
    }
}

// single excitation P -> A out of ket D
template <int KIND, int W>
__device__ double single_element(const DevSys &s, const uint64_t (&D)[W], int P, int A)
{
    const double sign = parity_between<W>(D, P, A);
    if constexpr (KIND == K_HUBBARD) {
        if ((P & 1) != (A & 1)) return 0.0;
        const int p = P >> 1, a = A >> 1, n = s.n_spatial;
        const int d = p > a ? p - a : a - p;
        const bool nb = (d == 1) || (s.periodic && d == n - 1);
        return nb ? (-s.t) * sign : 0.0;
    } else if constexpr (KIND == K_UEG) {
        return 0.0;
    } else {
        if ((P & 1) != (A & 1)) return 0.0;
        const int p = P >> 1, a = A >> 1, n = s.n_spatial;
        double v = s.h1[(size_t)a * n + p];
        for_bits<W>(D, [&](int Q) {
            if (Q != P) {
                const int q = Q >> 1;
                const double x = eri_at(s, a, p, q, q);
                const double y = ((A & 1) == (Q & 1)) ? eri_at(s, a, q, q, p) : 0.0;
                v = v + (x - y);
            }
        });
        return sign * v;
    }
}

// double excitation: holes P < Q, particles A < B, paired P -> A, Q -> B
template <int KIND, int W>
__device__ __forceinline__ double double_element(const DevSys &s, const uint64_t (&D)[W], int P, int Q, int A,
                                                 int B)
{
    uint64_t tmp[W];
#pragma unroll
    for (int i = 0; i < W; ++i) tmp[i] = D[i];
    const double s1 = parity_between<W>(tmp, P, A);
    flipbit<W>(tmp, P);
    flipbit<W>(tmp, A);
    const double s2 = parity_between<W>(tmp, Q, B);
    return (s1 * s2) * antisym<KIND>(s, A, B, P, Q);
}

// <bra|H|ket> for bra at most doubly excited from ket (else 0)
template <int KIND, int W>
__device__ double hij(const DevSys &s, const uint64_t (&bra)[W], const uint64_t (&ket)[W])
{
    int nd = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) nd += __popcll(bra[i] ^ ket[i]);
    if (nd == 0) return diag_element<KIND, W>(s, ket);
    if (nd != 2 && nd != 4) return 0.0;
    uint64_t hm[W], pm[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        hm[i] = ket[i] & ~bra[i];
        pm[i] = bra[i] & ~ket[i];
    }
    if (nd == 2) return single_element<KIND, W>(s, ket, select_bit<W>(hm, 0), select_bit<W>(pm, 0));
    return double_element<KIND, W>(s, ket, select_bit<W>(hm, 0), select_bit<W>(hm, 1), select_bit<W>(pm, 0),
                                   select_bit<W>(pm, 1));
}

// ---------------------------------------------------------------------------
// Excitation generators. Each returns true with the child, p_gen and H_child,D.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t even_bits(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// Hubbard chain: uniform over valid nearest-neighbour hops, in the order
// right-alpha, left-alpha, right-beta, left-beta, each by ascending site.
template <int W>
__device__ bool gen_hubbard(const DevSys &s, const uint64_t (&D)[W], uint32_t w0, uint64_t (&child)[W],
                            double &pgen, double &h)
{
    const int n = s.n_spatial;
    const uint32_t full = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1);
    uint32_t grp[4];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        const uint32_t m = even_bits(D[0] >> sg);
        uint32_t nxt, prv;
        if (s.periodic) {
            nxt = ((m >> 1) | ((m & 1u) << (n - 1))) & full;
            prv = ((m << 1) | (m >> (n - 1))) & full;
        } else {
            nxt = m >> 1;
            prv = (m << 1) & full;
        }
        uint32_t R = m & ~nxt, L = m & ~prv;
        if (!s.periodic) {
            R &= ~(1u << (n - 1));
            L &= ~1u;
        }
        grp[2 * sg] = R;
        grp[2 * sg + 1] = L;
    }
    const int c0 = __popc(grp[0]), c1 = __popc(grp[1]), c2 = __popc(grp[2]), c3 = __popc(grp[3]);
    const int nv = c0 + c1 + c2 + c3;
    if (nv == 0) return false;
    int k = (int)pick(w0, (uint32_t)nv);
    int g = 0;
    if (k >= c0) { k -= c0; g = 1;
        if (k >= c1) { k -= c1; g = 2;
            if (k >= c2) { k -= c2; g = 3; } } }
    const int p = select_in_word((uint64_t)grp[g], k);
    const int sg = g >> 1;
    const int q = (g & 1) ? (p + n - 1) % n : (p + 1) % n;
    const int P = 2 * p + sg, A = 2 * q + sg;
#pragma unroll
    for (int i = 0; i < W; ++i) child[i] = D[i];
    flipbit<W>(child, P);
    flipbit<W>(child, A);
    pgen = 1.0 / (double)nv;
    h = single_element<K_HUBBARD, W>(s, D, P, A);
    return true;
}

// UEG: uniform pair of occupied spin-orbitals, uniform A (same spin as the
// pair, or any spin for an opposite-spin pair), B fixed by momentum.
template <int W>
__device__ bool gen_ueg(const UegTables &s, const uint64_t (&D)[W], uint32_t w0, uint32_t w1,
                        uint64_t (&child)[W], double &pgen, double &h)
{
    const int N = s.nel;
    const uint32_t npairs = (uint32_t)(N * (N - 1) / 2);
    const int k = (int)pick(w0, npairs);
    // lexicographic unranking: i is the largest with i (2N - i - 1) / 2 <= k
    // (square-root estimate, then an exact integer correction)
    const float bb = (float)(2 * N - 1);
    int i = (int)((bb - sqrtf(bb * bb - 8.0f * (float)k)) * 0.5f);
    i = i < 0 ? 0 : (i > N - 2 ? N - 2 : i);
    while (i > 0 && i * (2 * N - i - 1) / 2 > k) --i;
    while (i < N - 2 && (i + 1) * (2 * N - i - 2) / 2 <= k) ++i;
    const int j = i + 1 + (k - i * (2 * N - i - 1) / 2);
    const int P = select_bit<W>(D, i), Q = select_bit<W>(D, j);
    const int sP = P & 1, sQ = Q & 1, M = s.M;
    int A;
    if (sP == sQ)
        A = 2 * (int)pick(w1, (uint32_t)M) + sP;
    else
        A = (int)pick(w1, (uint32_t)(2 * M));
    const int sA = A & 1, sB = sP + sQ - sA;
    const int p = P >> 1, q = Q >> 1, a = A >> 1;
    const int32_t bp = s.npk[p] + s.npk[q] - s.npk[a];
    const int bx = pk_comp(bp, 0), by = pk_comp(bp, 1), bz = pk_comp(bp, 2);
    const int g = s.gmax;
    if (bx < -g || bx > g || by < -g || by > g || bz < -g || bz > g) return false;
    const int b = s.grid[((bx + g) * s.gdim + (by + g)) * s.gdim + (bz + g)];
    if (b < 0) return false;
    const int B = 2 * b + sB;
    if (A == B || getbit<W>(D, A) || getbit<W>(D, B)) return false;
    const int lo = A < B ? A : B, hi = A < B ? B : A;
#pragma unroll
    for (int t = 0; t < W; ++t) child[t] = D[t];
    flipbit<W>(child, P);
    flipbit<W>(child, Q);
    flipbit<W>(child, lo);
    flipbit<W>(child, hi);
    pgen = sP == sQ ? s.pgen_same : s.pgen_opp;  // 2 / (C(N,2) n_A), n_A = M or 2M
    uint64_t tmp[W];
#pragma unroll
    for (int t2 = 0; t2 < W; ++t2) tmp[t2] = D[t2];
    const double s1 = parity_between<W>(tmp, P, lo);
    flipbit<W>(tmp, P);
    flipbit<W>(tmp, lo);
    const double s2 = parity_between<W>(tmp, Q, hi);
    h = (s1 * s2) * antisym_ueg(s, lo, hi, P, Q);
    return true;
}

// Heat-bath doubles (weights |<AB||PQ>| tabulated per pair) with uniform
// singles taken with probability p_single. The double branch uses a second
// Philox block, drawn only when needed.
template <int W>
__device__ bool gen_heatbath(const DevSys &s, double p_single, const uint64_t (&D)[W], const U4 &r0,
                             uint32_t attempt, uint32_t t, uint64_t hsh, uint32_t k0, uint32_t k1,
                             uint64_t (&child)[W], double &pgen, double &h, const double *stri = nullptr)
{
    // pair weights S_PQ: the full table, or (stri) its strict upper triangle
    // row by row, P*(2n-P-1)/2 + Q-P-1, as staged in LDS by the spawn kernel
    const int nso = s.n_so;
    auto spq = [&](int P, int Q) -> double {
        return stri ? stri[P * (2 * nso - P - 1) / 2 + (Q - P - 1)] : s.hb_S[P * nso + Q];
    };
    const int N = s.nel;
    const int n = s.n_so;
    const double d = u53(r0.x, r0.y);
    if (d < p_single) {
        const int e = (int)pick(r0.z, (uint32_t)N);
        const int P = select_bit<W>(D, e);
        const int sg = P & 1;
        const int nvirt = s.n_spatial - (sg ? s.nb : s.na);
        if (nvirt <= 0) return false;
        const int a = (int)pick(r0.w, (uint32_t)nvirt);
        uint64_t em[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            em[i] = ~D[i] & (sg ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull) & range_mask(i, 0, n);
        const int A = select_bit<W>(em, a);
        if (A < 0) return false;
#pragma unroll
        for (int i = 0; i < W; ++i) child[i] = D[i];
        flipbit<W>(child, P);
        flipbit<W>(child, A);
        pgen = p_single / (double)((int64_t)N * nvirt);
        h = single_element<K_MOLECULAR, W>(s, D, P, A);
        return true;
    }
    double T = 0.0;
    for_pairs<W>(D, [&](int P, int Q) { T = T + spq(P, Q); });
    if (!(T > 0.0)) return false;
    const U4 r1 = draw(TAG_SELECT2, attempt, t, hsh, k0, k1);
    const double x = u53(r1.x, r1.y) * T;
    double cum = 0.0;
    int Ps = -1, Qs = -1;
    for_pairs<W>(D, [&](int P, int Q) {
        if (Ps < 0) {
            cum = cum + spq(P, Q);
            if (x < cum) {
                Ps = P;
                Qs = Q;
            }
        }
    });
    if (Ps < 0) return false;
    const int64_t off = s.hb_off[Ps * n + Qs];
    const int cnt = s.hb_cnt[Ps * n + Qs];
    const double S = s.hb_S[Ps * n + Qs];
    const double y = u53(r1.z, r1.w) * S;
    // first entry with y < cdf (cdf is non-decreasing)
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (y < s.hb_cdf[off + mid]) hi = mid; else lo = mid + 1;
    }
    if (lo >= cnt) return false;
    const uint16_t ab = s.hb_AB[off + lo];
    const int A = ab & 0xFF, B = ab >> 8;
    if (getbit<W>(D, A) || getbit<W>(D, B)) return false;
#pragma unroll
    for (int i = 0; i < W; ++i) child[i] = D[i];
    flipbit<W>(child, Ps);
    flipbit<W>(child, Qs);
    flipbit<W>(child, A);
    flipbit<W>(child, B);
    h = double_element<K_MOLECULAR, W>(s, D, Ps, Qs, A, B);
    pgen = ((1.0 - p_single) * fabs(antisym<K_MOLECULAR>(s, A, B, Ps, Qs))) / T;
    return true;
}

}  // namespace fq
