/*
 * FCIQMC oracle (test infrastructure only; see fq_oracle.h).
 *
 * Plain single-threaded C, FP64 throughout, built with -ffp-contract=off so
 * that every product and sum is rounded exactly as written. Lists are sorted
 * arrays compared as unsigned big integers; spawned walkers are sorted with
 * qsort and merged with a two-pointer walk. Nothing here is blocked, fused or
 * reordered beyond the order each step states.
 */
#include "fq_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11). The paper's code   */
/* uses dSFMT (Sec. 3.1); a counter-based generator keyed by (seed, replica)  */
/* with counter (tag|attempt, iteration, det hash) makes every draw a pure    */
/* function of what it is used for, so list order never changes results.    */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u; /* Weyl increments of the Philox key schedule */
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0,1) from two words: top 32 bits from a, 21 from b. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * 0x1p-53;
}

/* floor(w * n / 2^32): an integer in [0, n) from one 32-bit word. */
static uint32_t pick(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

enum { TAG_SELECT = 0, TAG_SELECT2 = 1, TAG_SPAWN_ROUND = 2, TAG_DEATH = 3, TAG_SEMISTOCH = 4, TAG_CLUSTER = 5 };

static void draw(const or_run *r, uint32_t tag, uint32_t attempt, uint32_t t, uint64_t h,
                 uint32_t out[4]);

/* ------------------------------------------------------------------------- */
/* Determinant hash. The paper hashes bit strings with MurmurHash2 (Sec. 3.1, */
/* appendix "Parallelization", eq. hash). MurmurHash64A (Appleby, public      */
/* domain) over the 8W bytes of the words, least significant word first.     */
/* ------------------------------------------------------------------------- */
#define OR_HASH_SEED 0x9E3779B97F4A7C15ull

uint64_t or_hash64(const uint64_t *w, int W)
{
    const uint64_t m = 0xc6a4a7935bd1e995ull;
    const int r = 47;
    uint64_t h = OR_HASH_SEED ^ ((uint64_t)(8 * W) * m);
    for (int i = 0; i < W; ++i) {
        uint64_t k = w[i];
        k *= m;
        k ^= k >> r;
        k *= m;
        h ^= k;
        h *= m;
    }
    h ^= h >> r;
    h *= m;
    h ^= h >> r;
    return h;
}

/* ------------------------------------------------------------------------- */
/* Bit strings. Spin-orbital P = 2p + sigma (sigma 0 = alpha, 1 = beta) lives */
/* in word P/64, bit P%64. |D> = a+_{P1} a+_{P2} ... |0> with P1 < P2 < ...   */
/* ------------------------------------------------------------------------- */
static int getbit(const uint64_t *k, int P) { return (int)((k[P >> 6] >> (P & 63)) & 1u); }
static void setbit(uint64_t *k, int P) { k[P >> 6] |= (uint64_t)1 << (P & 63); }
static void clrbit(uint64_t *k, int P) { k[P >> 6] &= ~((uint64_t)1 << (P & 63)); }

static int occ_list(const uint64_t *k, int n_so, int *occ)
{
    int n = 0;
    for (int P = 0; P < n_so; ++P)
        if (getbit(k, P)) occ[n++] = P;
    return n;
}

static int key_cmp(const uint64_t *a, const uint64_t *b, int W)
{
    for (int i = W - 1; i >= 0; --i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

/* (-1)^{number of occupied spin-orbitals strictly between P and A} */
static double parity_between(const uint64_t *k, int P, int A)
{
    int lo = P < A ? P : A, hi = P < A ? A : P, c = 0;
    for (int X = lo + 1; X < hi; ++X) c += getbit(k, X);
    return (c & 1) ? -1.0 : 1.0;
}

/* ------------------------------------------------------------------------- */
/* Systems (paper Sec. 4.3: UEG and Hubbard model systems; Sec. 3.1 and the   */
/* tutorial appendix: molecular integrals h_pq, (pq|rs)).                     */
/* ------------------------------------------------------------------------- */
struct or_sys {
    int kind, n_spatial, n_so, W, nel, na, nb;
    /* Hubbard ring / chain */
    int periodic;
    double t, U;
    /* uniform electron gas */
    double rs, L, k2, vc;
    int ecut, vlen, gmax, gdim;
    int32_t *nvec;  /* [n_spatial][3] */
    double *eps;    /* kinetic energy per spatial orbital */
    double *vtab;   /* v(|dn|^2) */
    int32_t *grid;  /* momentum -> spatial index, -1 outside the basis */
    /* molecular */
    double *h1, *eri;
    /* heat-bath tables, pair index P*n_so + Q for P < Q */
    int64_t *hb_off;
    int32_t *hb_cnt;
    double *hb_S;
    int32_t *hb_A, *hb_B;
    double *hb_cdf;
    int64_t hb_n;
    uint64_t ref[OR_MAXW];
    double H00;
};

static or_sys *sys_alloc(int kind, int n_spatial, int na, int nb)
{
    or_sys *s = (or_sys *)calloc(1, sizeof(or_sys));
    s->kind = kind;
    s->n_spatial = n_spatial;
    s->n_so = 2 * n_spatial;
    s->W = (s->n_so + 63) / 64;
    s->na = na;
    s->nb = nb;
    s->nel = na + nb;
    return s;
}

static double eri_at(const or_sys *s, int p, int q, int r, int t)
{
    int n = s->n_spatial;
    return s->eri[(((size_t)p * n + q) * n + r) * n + t];
}

static int dn2(const or_sys *s, int p, int q)
{
    int d = 0;
    for (int c = 0; c < 3; ++c) {
        int x = s->nvec[3 * p + c] - s->nvec[3 * q + c];
        d += x * x;
    }
    return d;
}

/* ---- Slater-Condon rules, diagonal ---- */
double or_diag(const or_sys *s, const uint64_t *key)
{
    int occ[1024];
    int n = occ_list(key, s->n_so, occ);
    double e = 0.0;
    if (s->kind == OR_HUBBARD) {
        for (int p = 0; p < s->n_spatial; ++p)
            if (getbit(key, 2 * p) && getbit(key, 2 * p + 1)) e = e + s->U;
        return e;
    }
    if (s->kind == OR_UEG) {
        for (int i = 0; i < n; ++i) e = e + s->eps[occ[i] >> 1];
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if ((occ[i] & 1) == (occ[j] & 1)) e = e - s->vtab[dn2(s, occ[i] >> 1, occ[j] >> 1)];
        return e;
    }
    for (int i = 0; i < n; ++i) {
        int p = occ[i] >> 1;
        e = e + s->h1[(size_t)p * s->n_spatial + p];
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int p = occ[i] >> 1, q = occ[j] >> 1;
            double x = eri_at(s, p, p, q, q);
            double y = ((occ[i] & 1) == (occ[j] & 1)) ? eri_at(s, p, q, q, p) : 0.0;
            e = e + (x - y);
        }
    return e;
}

/* ---- single excitation P -> A out of ket D (A empty, P occupied in D) ---- */
static double single_element(const or_sys *s, const uint64_t *D, int P, int A)
{
    double sign = parity_between(D, P, A);
    if (s->kind == OR_HUBBARD) {
        if ((P & 1) != (A & 1)) return 0.0;
        int p = P >> 1, a = A >> 1, n = s->n_spatial;
        int d = p > a ? p - a : a - p;
        int nb = (d == 1) || (s->periodic && d == n - 1);
        return nb ? (-s->t) * sign : 0.0;
    }
    if (s->kind == OR_UEG) return 0.0; /* momentum conservation */
    if ((P & 1) != (A & 1)) return 0.0;
    int occ[1024];
    int n = occ_list(D, s->n_so, occ);
    int p = P >> 1, a = A >> 1;
    double v = s->h1[(size_t)a * s->n_spatial + p];
    for (int i = 0; i < n; ++i) {
        int Q = occ[i];
        if (Q == P) continue;
        int q = Q >> 1;
        double x = eri_at(s, a, p, q, q);
        double y = ((A & 1) == (Q & 1)) ? eri_at(s, a, q, q, p) : 0.0;
        v = v + (x - y);
    }
    return sign * v;
}

/* <AB|PQ> - <AB|QP> in physicists' notation with spin-orbital indices */
static double antisym(const or_sys *s, int A, int B, int P, int Q)
{
    int sa = A & 1, sb = B & 1, sp = P & 1, sq = Q & 1;
    int a = A >> 1, b = B >> 1, p = P >> 1, q = Q >> 1;
    if (s->kind == OR_HUBBARD) return 0.0; /* on-site U is diagonal only */
    if (s->kind == OR_UEG) {
        for (int c = 0; c < 3; ++c)
            if (s->nvec[3 * a + c] + s->nvec[3 * b + c] != s->nvec[3 * p + c] + s->nvec[3 * q + c])
                return 0.0;
        double x = (sa == sp && sb == sq) ? s->vtab[dn2(s, p, a)] : 0.0;
        double y = (sa == sq && sb == sp) ? s->vtab[dn2(s, q, a)] : 0.0;
        return x - y;
    }
    double x = (sa == sp && sb == sq) ? eri_at(s, a, p, b, q) : 0.0;
    double y = (sa == sq && sb == sp) ? eri_at(s, a, q, b, p) : 0.0;
    return x - y;
}

/* ---- double excitation: holes P < Q, particles A < B, paired P->A, Q->B ---- */
static double double_element(const or_sys *s, const uint64_t *D, int P, int Q, int A, int B)
{
    uint64_t tmp[OR_MAXW];
    memcpy(tmp, D, sizeof(uint64_t) * s->W);
    double s1 = parity_between(tmp, P, A);
    clrbit(tmp, P);
    setbit(tmp, A);
    double s2 = parity_between(tmp, Q, B);
    return (s1 * s2) * antisym(s, A, B, P, Q);
}

double or_hij(const or_sys *s, const uint64_t *bra, const uint64_t *ket)
{
    int nd = 0;
    for (int i = 0; i < s->W; ++i) nd += __builtin_popcountll(bra[i] ^ ket[i]);
    if (nd == 0) return or_diag(s, ket);
    if (nd != 2 && nd != 4) return 0.0;
    int holes[2], parts[2], nh = 0, np = 0;
    for (int X = 0; X < s->n_so; ++X) {
        int kb = getbit(ket, X), bb = getbit(bra, X);
        if (kb && !bb) holes[nh++] = X;
        if (bb && !kb) parts[np++] = X;
    }
    if (nh != np) return 0.0;
    if (nh == 1) return single_element(s, ket, holes[0], parts[0]);
    return double_element(s, ket, holes[0], holes[1], parts[0], parts[1]);
}

static void finish_sys(or_sys *s)
{
    s->H00 = or_diag(s, s->ref);
}

or_sys *or_hubbard_new(int n_sites, int periodic, double t, double U, int n_alpha, int n_beta)
{
    if (n_sites < 3 || 2 * n_sites > 64 * OR_MAXW || n_alpha > n_sites || n_beta > n_sites ||
        n_alpha < 0 || n_beta < 0)
        return NULL;
    or_sys *s = sys_alloc(OR_HUBBARD, n_sites, n_alpha, n_beta);
    s->periodic = periodic;
    s->t = t;
    s->U = U;
    /* reference: alpha on sites 0,2,4,... then 1,3,...; beta on 1,3,5,... then 0,2,... */
    int placed = 0;
    for (int pass = 0; pass < 2 && placed < n_alpha; ++pass)
        for (int p = pass; p < n_sites && placed < n_alpha; p += 2, ++placed) setbit(s->ref, 2 * p);
    placed = 0;
    for (int pass = 1; pass >= 0 && placed < n_beta; --pass)
        for (int p = pass; p < n_sites && placed < n_beta; p += 2, ++placed) setbit(s->ref, 2 * p + 1);
    finish_sys(s);
    return s;
}

typedef struct { int n2, x, y, z; } pw_t;
static int pw_cmp(const void *a, const void *b)
{
    const pw_t *u = (const pw_t *)a, *v = (const pw_t *)b;
    if (u->n2 != v->n2) return u->n2 - v->n2;
    if (u->x != v->x) return u->x - v->x;
    if (u->y != v->y) return u->y - v->y;
    return u->z - v->z;
}

/* Plane waves n in Z^3 with |n|^2 <= ecut in a simple-cubic box of side
 * L = rs * cbrt(4 pi N / 3); kinetic (2pi/L)^2 |n|^2 / 2; Coulomb
 * v(q) = 4 pi / (L^3 |k_q|^2), q = 0 excluded (paper Sec. 4.3, UEG). */
or_sys *or_ueg_new(double rs, int ecut_n2, int n_alpha, int n_beta)
{
    int c = 0;
    while ((c + 1) * (c + 1) <= ecut_n2) ++c;
    int side = 2 * c + 1;
    pw_t *pw = (pw_t *)malloc(sizeof(pw_t) * (size_t)side * side * side);
    int m = 0;
    for (int x = -c; x <= c; ++x)
        for (int y = -c; y <= c; ++y)
            for (int z = -c; z <= c; ++z) {
                int n2 = x * x + y * y + z * z;
                if (n2 <= ecut_n2) {
                    pw[m].n2 = n2; pw[m].x = x; pw[m].y = y; pw[m].z = z;
                    ++m;
                }
            }
    qsort(pw, (size_t)m, sizeof(pw_t), pw_cmp);
    if (2 * m > 64 * OR_MAXW || n_alpha > m || n_beta > m) { free(pw); return NULL; }
    or_sys *s = sys_alloc(OR_UEG, m, n_alpha, n_beta);
    s->rs = rs;
    s->ecut = ecut_n2;
    s->nvec = (int32_t *)malloc(sizeof(int32_t) * 3 * m);
    s->eps = (double *)malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) {
        s->nvec[3 * i] = pw[i].x; s->nvec[3 * i + 1] = pw[i].y; s->nvec[3 * i + 2] = pw[i].z;
    }
    double N = (double)(n_alpha + n_beta);
    s->L = rs * cbrt((4.0 * M_PI * N) / 3.0);
    double g = (2.0 * M_PI) / s->L;
    s->k2 = g * g;
    s->vc = (4.0 * M_PI) / ((s->L * s->L) * s->L);
    for (int i = 0; i < m; ++i) s->eps[i] = (s->k2 * (double)pw[i].n2) * 0.5;
    s->vlen = 4 * ecut_n2 + 1;
    s->vtab = (double *)malloc(sizeof(double) * s->vlen);
    s->vtab[0] = 0.0;
    for (int d = 1; d < s->vlen; ++d) s->vtab[d] = s->vc / (s->k2 * (double)d);
    s->gmax = 3 * c;
    s->gdim = 2 * s->gmax + 1;
    size_t gsz = (size_t)s->gdim * s->gdim * s->gdim;
    s->grid = (int32_t *)malloc(sizeof(int32_t) * gsz);
    for (size_t i = 0; i < gsz; ++i) s->grid[i] = -1;
    for (int i = 0; i < m; ++i) {
        size_t gi = ((size_t)(pw[i].x + s->gmax) * s->gdim + (pw[i].y + s->gmax)) * s->gdim +
                    (pw[i].z + s->gmax);
        s->grid[gi] = i;
    }
    free(pw);
    for (int i = 0; i < n_alpha; ++i) setbit(s->ref, 2 * i);
    for (int i = 0; i < n_beta; ++i) setbit(s->ref, 2 * i + 1);
    finish_sys(s);
    return s;
}

static int ueg_lookup(const or_sys *s, int x, int y, int z)
{
    if (x < -s->gmax || x > s->gmax || y < -s->gmax || y > s->gmax || z < -s->gmax || z > s->gmax)
        return -1;
    return s->grid[((size_t)(x + s->gmax) * s->gdim + (y + s->gmax)) * s->gdim + (z + s->gmax)];
}

/* Heat-bath tables for doubles (paper Sec. 2.1 and 4.1: heat-bath excitation
 * generation): for each spin-orbital pair P < Q the allowed A < B (spin
 * conserving, A,B not in {P,Q}) in lexicographic order with weight
 * |<AB|PQ> - <AB|QP>|, and their sequential running sum. */
static void build_heatbath(or_sys *s)
{
    int n = s->n_so;
    s->hb_off = (int64_t *)calloc((size_t)n * n, sizeof(int64_t));
    s->hb_cnt = (int32_t *)calloc((size_t)n * n, sizeof(int32_t));
    s->hb_S = (double *)calloc((size_t)n * n, sizeof(double));
    int64_t total = 0;
    for (int P = 0; P < n; ++P)
        for (int Q = P + 1; Q < n; ++Q) {
            int cnt = 0;
            for (int A = 0; A < n; ++A)
                for (int B = A + 1; B < n; ++B) {
                    if (A == P || A == Q || B == P || B == Q) continue;
                    if ((A & 1) + (B & 1) != (P & 1) + (Q & 1)) continue;
                    ++cnt;
                }
            s->hb_off[P * n + Q] = total;
            s->hb_cnt[P * n + Q] = cnt;
            total += cnt;
        }
    s->hb_n = total;
    s->hb_A = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    s->hb_B = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    s->hb_cdf = (double *)malloc(sizeof(double) * (size_t)total);
    for (int P = 0; P < n; ++P)
        for (int Q = P + 1; Q < n; ++Q) {
            int64_t e = s->hb_off[P * n + Q];
            double c = 0.0;
            for (int A = 0; A < n; ++A)
                for (int B = A + 1; B < n; ++B) {
                    if (A == P || A == Q || B == P || B == Q) continue;
                    if ((A & 1) + (B & 1) != (P & 1) + (Q & 1)) continue;
                    double w = fabs(antisym(s, A, B, P, Q));
                    c = c + w;
                    s->hb_A[e] = A;
                    s->hb_B[e] = B;
                    s->hb_cdf[e] = c;
                    ++e;
                }
            s->hb_S[P * n + Q] = c;
        }
}

or_sys *or_molecular_new(int n_orb, const double *h1, const double *eri, int n_alpha, int n_beta)
{
    if (n_orb <= 0 || 2 * n_orb > 64 * OR_MAXW || n_alpha > n_orb || n_beta > n_orb) return NULL;
    or_sys *s = sys_alloc(OR_MOLECULAR, n_orb, n_alpha, n_beta);
    size_t n2 = (size_t)n_orb * n_orb;
    s->h1 = (double *)malloc(sizeof(double) * n2);
    s->eri = (double *)malloc(sizeof(double) * n2 * n2);
    memcpy(s->h1, h1, sizeof(double) * n2);
    memcpy(s->eri, eri, sizeof(double) * n2 * n2);
    for (int i = 0; i < n_alpha; ++i) setbit(s->ref, 2 * i);
    for (int i = 0; i < n_beta; ++i) setbit(s->ref, 2 * i + 1);
    build_heatbath(s);
    finish_sys(s);
    return s;
}

void or_sys_free(or_sys *s)
{
    if (!s) return;
    free(s->nvec); free(s->eps); free(s->vtab); free(s->grid);
    free(s->h1); free(s->eri);
    free(s->hb_off); free(s->hb_cnt); free(s->hb_S); free(s->hb_A); free(s->hb_B); free(s->hb_cdf);
    free(s);
}

void or_sys_info(const or_sys *s, int32_t *iout, double *dout)
{
    iout[0] = s->kind; iout[1] = s->n_spatial; iout[2] = s->n_so; iout[3] = s->W;
    iout[4] = s->nel; iout[5] = s->na; iout[6] = s->nb;
    dout[0] = s->H00; dout[1] = s->L; dout[2] = s->k2; dout[3] = s->vc;
}

void or_sys_reference(const or_sys *s, uint64_t *key) { memcpy(key, s->ref, sizeof(uint64_t) * s->W); }

void or_ueg_orbitals(const or_sys *s, int32_t *nvec)
{
    if (s->nvec) memcpy(nvec, s->nvec, sizeof(int32_t) * 3 * s->n_spatial);
}

int64_t or_heatbath_size(const or_sys *s) { return s->hb_n; }

/* ------------------------------------------------------------------------- */
/* Excitation generators ("system-dependent", Sec. 2.4).                     */
/* ------------------------------------------------------------------------- */

/* Hubbard: uniform over the valid nearest-neighbour hops of either spin. */
static int gen_hubbard(const or_sys *s, const uint64_t *D, const uint32_t *w, uint64_t *child,
                       double *pgen, double *hij)
{
    int n = s->n_spatial;
    /* candidate hops in the order: right-alpha, left-alpha, right-beta, left-beta, ascending site */
    int from[256], to[256], nv = 0;
    for (int sg = 0; sg < 2; ++sg)
        for (int dir = 0; dir < 2; ++dir)
            for (int p = 0; p < n; ++p) {
                int q;
                if (dir == 0) {
                    if (p == n - 1 && !s->periodic) continue;
                    q = (p + 1) % n;
                } else {
                    if (p == 0 && !s->periodic) continue;
                    q = (p + n - 1) % n;
                }
                if (getbit(D, 2 * p + sg) && !getbit(D, 2 * q + sg)) {
                    from[nv] = 2 * p + sg;
                    to[nv] = 2 * q + sg;
                    ++nv;
                }
            }
    if (nv == 0) return 0;
    uint32_t k = pick(w[0], (uint32_t)nv);
    int P = from[k], A = to[k];
    memcpy(child, D, sizeof(uint64_t) * s->W);
    clrbit(child, P);
    setbit(child, A);
    *pgen = 1.0 / (double)nv;
    *hij = single_element(s, D, P, A);
    return 1;
}

/* pair index k in [0, C(N,2)) -> (i, j), i < j, lexicographic */
static void unrank_pair(int N, uint32_t k, int *i, int *j)
{
    int a = 0;
    uint32_t rem = k;
    while (rem >= (uint32_t)(N - 1 - a)) { rem -= (uint32_t)(N - 1 - a); ++a; }
    *i = a;
    *j = a + 1 + (int)rem;
}

/* UEG: uniform pair of occupied spin-orbitals, uniform A, B by momentum. */
static int gen_ueg(const or_sys *s, const uint64_t *D, const uint32_t *w, uint64_t *child,
                   double *pgen, double *hij)
{
    int occ[1024];
    int N = occ_list(D, s->n_so, occ);
    uint32_t npairs = (uint32_t)(N * (N - 1) / 2);
    int i, j;
    unrank_pair(N, pick(w[0], npairs), &i, &j);
    int P = occ[i], Q = occ[j];
    int sP = P & 1, sQ = Q & 1, M = s->n_spatial, A, na;
    if (sP == sQ) {
        na = M;
        A = 2 * (int)pick(w[1], (uint32_t)M) + sP;
    } else {
        na = 2 * M;
        A = (int)pick(w[1], (uint32_t)(2 * M));
    }
    int sA = A & 1, sB = sP + sQ - sA;
    int p = P >> 1, q = Q >> 1, a = A >> 1;
    int bx = s->nvec[3 * p] + s->nvec[3 * q] - s->nvec[3 * a];
    int by = s->nvec[3 * p + 1] + s->nvec[3 * q + 1] - s->nvec[3 * a + 1];
    int bz = s->nvec[3 * p + 2] + s->nvec[3 * q + 2] - s->nvec[3 * a + 2];
    int b = ueg_lookup(s, bx, by, bz);
    if (b < 0) return 0;
    int B = 2 * b + sB;
    if (A == B || getbit(D, A) || getbit(D, B)) return 0;
    int lo = A < B ? A : B, hi = A < B ? B : A;
    memcpy(child, D, sizeof(uint64_t) * s->W);
    clrbit(child, P); clrbit(child, Q); setbit(child, lo); setbit(child, hi);
    *pgen = 2.0 / (double)((int64_t)npairs * na);
    *hij = double_element(s, D, P, Q, lo, hi);
    return 1;
}

/* Heat-bath doubles with uniform singles (paper Sec. 2.1 and 4.1). */
static int gen_heatbath(const or_sys *s, double p_single, const uint64_t *D, const uint32_t *w,
                        uint64_t *child, double *pgen, double *hij)
{
    int occ[1024];
    int N = occ_list(D, s->n_so, occ);
    int n = s->n_so;
    double d = u53(w[0], w[1]);
    if (d < p_single) {
        int P = occ[pick(w[2], (uint32_t)N)];
        int sg = P & 1;
        int nel_s = sg ? s->nb : s->na;
        int nvirt = s->n_spatial - nel_s;
        if (nvirt <= 0) return 0;
        uint32_t a = pick(w[3], (uint32_t)nvirt);
        int A = -1;
        uint32_t seen = 0;
        for (int X = sg; X < n; X += 2)
            if (!getbit(D, X)) {
                if (seen == a) { A = X; break; }
                ++seen;
            }
        if (A < 0) return 0;
        memcpy(child, D, sizeof(uint64_t) * s->W);
        clrbit(child, P);
        setbit(child, A);
        *pgen = p_single / (double)((int64_t)N * nvirt);
        *hij = single_element(s, D, P, A);
        return 1;
    }
    double T = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) T = T + s->hb_S[occ[i] * n + occ[j]];
    if (!(T > 0.0)) return 0;
    double u = u53(w[4], w[5]);
    double x = u * T, cum = 0.0;
    int P = -1, Q = -1;
    for (int i = 0; i < N && P < 0; ++i)
        for (int j = i + 1; j < N; ++j) {
            cum = cum + s->hb_S[occ[i] * n + occ[j]];
            if (x < cum) { P = occ[i]; Q = occ[j]; break; }
        }
    if (P < 0) return 0;
    int64_t off = s->hb_off[P * n + Q];
    int cnt = s->hb_cnt[P * n + Q];
    double S = s->hb_S[P * n + Q];
    double y = u53(w[6], w[7]) * S;
    int e = -1;
    for (int k = 0; k < cnt; ++k)
        if (y < s->hb_cdf[off + k]) { e = k; break; }
    if (e < 0) return 0;
    int A = s->hb_A[off + e], B = s->hb_B[off + e];
    if (getbit(D, A) || getbit(D, B)) return 0;
    double v = double_element(s, D, P, Q, A, B);
    memcpy(child, D, sizeof(uint64_t) * s->W);
    clrbit(child, P); clrbit(child, Q); setbit(child, A); setbit(child, B);
    *pgen = ((1.0 - p_single) * fabs(antisym(s, A, B, P, Q))) / T;
    *hij = v;
    return 1;
}

int or_exgen(const or_sys *s, int exgen, double p_single, const uint64_t *key, const uint32_t *w,
             uint64_t *child, double *pgen, double *hij)
{
    if (exgen == OR_EXGEN_HUB && s->kind == OR_HUBBARD) return gen_hubbard(s, key, w, child, pgen, hij);
    if (exgen == OR_EXGEN_UEG && s->kind == OR_UEG) return gen_ueg(s, key, w, child, pgen, hij);
    if (exgen == OR_EXGEN_HEATBATH && s->kind == OR_MOLECULAR)
        return gen_heatbath(s, p_single, key, w, child, pgen, hij);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The run: main list, one projector iteration per step.                     */
/* ------------------------------------------------------------------------- */
struct or_run {
    const or_sys *s;
    or_qmc q;
    int W;
    int64_t n, cap;
    uint64_t *keys;
    int32_t *pops;
    double *kdiag;
    int32_t *dslot;
    double S;
    int vary;
    int64_t nprev, t;
    int64_t cu, thr, target_units;
    uint32_t rkey[2];
    or_estimators est;
    /* spawned walkers of the last iteration */
    int64_t ns, scap;
    uint64_t *skeys;
    int32_t *samps;
    uint8_t *sinit;
    /* deterministic space */
    int ss_active;
    int64_t nd;
    uint64_t *dkeys;     /* D order */
    double *kdd;         /* nd x nd */
    uint64_t *dsorted;   /* sorted copy of the keys */
    int32_t *dsorted_ix; /* D index of each sorted key */
    double *last_y;
    /* time-step search (tutorial appendix: tau_search) */
    double rs_max;  /* largest |H_ji| / p_gen over the attempts so far */
    double kd_max;  /* largest K_ii over the entries of the last death step */
    int kd_any;
};

static void draw(const or_run *r, uint32_t tag, uint32_t attempt, uint32_t t, uint64_t h,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {(tag << 28) | attempt, t, (uint32_t)h, (uint32_t)(h >> 32)};
    or_philox4x32_10(ctr, r->rkey, out);
}

/* stochastic rounding of m >= 0 with uniform u: floor(m) + [u < m - floor(m)] */
static int64_t sround(double m, double u)
{
    double f = floor(m);
    int64_t k = (int64_t)f;
    if (u < m - f) k += 1;
    return k;
}

static void list_reserve(or_run *r, int64_t need)
{
    if (need <= r->cap) return;
    int64_t c = r->cap ? r->cap : 1024;
    while (c < need) c *= 2;
    r->keys = (uint64_t *)realloc(r->keys, sizeof(uint64_t) * (size_t)c * r->W);
    r->pops = (int32_t *)realloc(r->pops, sizeof(int32_t) * (size_t)c);
    r->kdiag = (double *)realloc(r->kdiag, sizeof(double) * (size_t)c);
    r->dslot = (int32_t *)realloc(r->dslot, sizeof(int32_t) * (size_t)c);
    r->cap = c;
}

static void push_spawn(or_run *r, const uint64_t *key, int32_t amp, uint8_t init)
{
    if (r->ns == r->scap) {
        r->scap = r->scap ? 2 * r->scap : 4096;
        r->skeys = (uint64_t *)realloc(r->skeys, sizeof(uint64_t) * (size_t)r->scap * r->W);
        r->samps = (int32_t *)realloc(r->samps, sizeof(int32_t) * (size_t)r->scap);
        r->sinit = (uint8_t *)realloc(r->sinit, (size_t)r->scap);
    }
    memcpy(r->skeys + (size_t)r->ns * r->W, key, sizeof(uint64_t) * r->W);
    r->samps[r->ns] = amp;
    r->sinit[r->ns] = init;
    r->ns++;
}

static int64_t dspace_find(const or_run *r, const uint64_t *key)
{
    int64_t lo = 0, hi = r->nd;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = key_cmp(r->dsorted + (size_t)mid * r->W, key, r->W);
        if (c == 0) return r->dsorted_ix[mid];
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

static int64_t n_attempts(const or_run *r, int32_t pop)
{
    int64_t a = pop < 0 ? -(int64_t)pop : (int64_t)pop;
    int b = r->q.fixed_point_bits;
    if (b == 0) return a;
    return (a + ((int64_t)1 << b) - 1) >> b;
}

static int is_reference(const or_run *r, const uint64_t *key) { return key_cmp(key, r->s->ref, r->W) == 0; }

/* Words of one determinant (s->W) in a key: the key itself for FCIQMC; for
 * the density-matrix methods the bra is the first half, the ket the second. */
static int det_words(const or_run *r) { return r->s->W; }

/* The diagonal element of an entry, relative to H_00, as death uses it.
 * FCIQMC: K_ii = H_ii - H_00.
 * DMQMC: the symmetrised Bloch equation (Sec. 2.3, eq. dmqmc) gives the pair
 *   (i, j) the diagonal (H_ii + H_jj) / 2: here (K_ii + K_jj) / 2.
 * IP-DMQMC (eq. ipdmqmc, H^0 the diagonal part of H): df/dtau = H^0 f - f H
 *   gives the pair (i, j) the diagonal H_jj - H^0_ii = K_jj - K_ii. */
static double entry_kdiag(const or_run *r, const uint64_t *key)
{
    const or_sys *s = r->s;
    if (r->q.method == OR_FCIQMC || r->q.method == OR_CCMC) return or_diag(s, key) - s->H00;
    int w = det_words(r);
    double ki = or_diag(s, key) - s->H00;
    double kj = or_diag(s, key + w) - s->H00;
    if (r->q.method == OR_DMQMC) return (ki + kj) * 0.5;
    return kj - ki;
}

/* Fixed-point accumulation of one FP64 term at resolution 2^-64, split into
 * four 32-bit limbs; the limb sums are exact and order independent. */
static void acc_term(int64_t limbs[4], double x)
{
    if (x == 0.0) return;
    int neg = x < 0.0;
    double a = neg ? -x : x;
    unsigned __int128 X = (unsigned __int128)(a * 0x1p64);
    for (int k = 0; k < 4; ++k) {
        int64_t l = (int64_t)(uint32_t)(X >> (32 * k));
        limbs[k] += neg ? -l : l;
    }
}

static double limbs_value(const int64_t limbs[4])
{
    __int128 tot = 0;
    for (int k = 0; k < 4; ++k) tot += (__int128)limbs[k] * ((__int128)1 << (32 * k));
    return (double)tot * 0x1p-64;
}

/* Projected energy (tutorial appendix): numerator sum_{j != 0} H_0j N_j
 * over the determinants at most doubly excited from D_0; N_0 as denominator.
 * Density-matrix methods (Sec. 2.3): the thermal energy Tr(rho H) / Tr(rho),
 * numerator sum over pairs of rho_ij H_ji (pairs at most doubly excited from
 * each other; H_ii on the diagonal), denominator the trace sum_i rho_ii. */
static void compute_estimators(or_run *r)
{
    or_estimators *e = &r->est;
    int64_t nw = 0, n0 = 0;
    int64_t limbs[4] = {0, 0, 0, 0}, plimbs[4] = {0, 0, 0, 0};
    int64_t n1 = 0;
    int64_t *singles = NULL;
    if (r->q.method == OR_CCMC) singles = (int64_t *)malloc(sizeof(int64_t) * (size_t)(r->n ? r->n : 1));
    int dm = r->q.method == OR_DMQMC || r->q.method == OR_IPDMQMC;
    int w = det_words(r);
    for (int64_t i = 0; i < r->n; ++i) {
        const uint64_t *k = r->keys + (size_t)i * r->W;
        int32_t p = r->pops[i];
        nw += p < 0 ? -(int64_t)p : p;
        if (dm) {
            int nd = 0;
            for (int x = 0; x < w; ++x) nd += __builtin_popcountll(k[x] ^ k[w + x]);
            if (nd == 0) {
                n0 += p;
                acc_term(limbs, or_diag(r->s, k) * (double)p);
            } else if (nd == 2 || nd == 4) {
                acc_term(limbs, or_hij(r->s, k + w, k) * (double)p);
            }
            continue;
        }
        if (is_reference(r, k)) { n0 = p; continue; }
        int nd = 0;
        for (int x = 0; x < r->W; ++x) nd += __builtin_popcountll(k[x] ^ r->s->ref[x]);
        if (singles && nd == 2 && p != 0) singles[n1++] = i;
        if (nd != 2 && nd != 4) continue;
        double h = or_hij(r->s, r->s->ref, k);
        acc_term(limbs, h * (double)p);
    }
    /* CCMC (Sec. 2.2): t~_j = <D_j|Psi> of a double also holds the products of
       pairs of singles, (1 / N_0) sgn N_a N_b for a_a a_b D_0 = sgn D_j; their
       part of sum_j H_0j t~_j is summed exactly here and divided by N_0 below */
    for (int64_t x = 0; x < n1; ++x)
        for (int64_t y = x + 1; y < n1; ++y) {
            uint64_t ex[2 * OR_MAXW], D[OR_MAXW];
            memcpy(ex, r->keys + (size_t)singles[x] * r->W, sizeof(uint64_t) * r->W);
            memcpy(ex + r->W, r->keys + (size_t)singles[y] * r->W, sizeof(uint64_t) * r->W);
            int sg = or_cluster_collapse(r->s, ex, 2, D);
            if (sg == 0) continue;
            /* H_0,ab (N_a N_b): the product of the pair first, so the term is
               the same whichever single comes first */
            double h = or_hij(r->s, r->s->ref, D);
            double term = h * ((double)r->pops[singles[x]] * (double)r->pops[singles[y]]);
            acc_term(plimbs, sg > 0 ? term : -term);
        }
    free(singles);
    e->iteration = r->t;
    e->n_walkers_units = nw;
    e->n_occupied = r->n;
    e->ref_pop_units = n0;
    memcpy(e->num_limbs, limbs, sizeof(limbs));
    memcpy(e->pair_limbs, plimbs, sizeof(plimbs));
    double num = limbs_value(limbs);
    if (r->q.method == OR_CCMC && n0 != 0) num = num + limbs_value(plimbs) / (double)n0;
    double scale = ldexp(1.0, -r->q.fixed_point_bits);
    e->proj_numerator = num * scale;
    e->proj_energy = n0 != 0 ? num / (double)n0 : NAN;
    e->shift = r->S;
    e->vary_shift = r->vary;
    e->e_ref = r->s->H00;
}

or_run *or_run_new(const or_sys *s, const or_qmc *q)
{
    /* b = 1, 2 would allow more than 2^28 attempts per determinant (the
       attempt index field of the random-number counter): refused */
    if (!s || !q || !(q->tau > 0.0) || q->fixed_point_bits < 0 || q->fixed_point_bits > 20 ||
        (q->fixed_point_bits > 0 && q->fixed_point_bits < 3) ||
        q->shift_period <= 0)
        return NULL;
    if (q->excit_gen == OR_EXGEN_HUB && s->kind != OR_HUBBARD) return NULL;
    if (q->excit_gen == OR_EXGEN_UEG && s->kind != OR_UEG) return NULL;
    if (q->excit_gen == OR_EXGEN_HEATBATH && s->kind != OR_MOLECULAR) return NULL;
    if (q->method < OR_FCIQMC || q->method > OR_CCMC) return NULL;
    /* CCMC: excitors of level 1..6 (clusters of at most 8 excitors), no
       initiator rule, deterministic space or time-step search */
    if (q->method == OR_CCMC && (q->ccmc_truncation < 1 || q->ccmc_truncation > 6 || q->initiator ||
                                 q->ss_size > 0 || q->tau_search))
        return NULL;
    /* density matrices: pairs of determinants of at most four words, no
       initiator rule, deterministic space or time-step search */
    if ((q->method == OR_DMQMC || q->method == OR_IPDMQMC) &&
        (2 * s->W > OR_MAXW || q->initiator || q->ss_size > 0 || q->tau_search))
        return NULL;
    or_run *r = (or_run *)calloc(1, sizeof(or_run));
    r->s = s;
    r->q = *q;
    r->W = (q->method == OR_FCIQMC || q->method == OR_CCMC) ? s->W : 2 * s->W;
    double scale = ldexp(1.0, q->fixed_point_bits);
    r->cu = q->fixed_point_bits ? (int64_t)floor(q->spawn_cutoff * scale + 0.5) : 0;
    r->thr = (int64_t)floor(q->initiator_threshold * scale);
    r->rkey[0] = (uint32_t)q->seed;
    r->rkey[1] = (uint32_t)(q->seed >> 32) ^ (uint32_t)q->replica_id;
    list_reserve(r, 1);
    /* the reference, or the pair (D_0, D_0) */
    memcpy(r->keys, s->ref, sizeof(uint64_t) * s->W);
    if (r->W != s->W) memcpy(r->keys + s->W, s->ref, sizeof(uint64_t) * s->W);
    r->pops[0] = (int32_t)floor(q->init_pop * scale + 0.5);
    r->kdiag[0] = entry_kdiag(r, r->keys);
    r->dslot[0] = -1;
    r->n = 1;
    r->S = q->initial_shift;
    compute_estimators(r);
    r->est.tau = r->q.tau;
    return r;
}

void or_run_free(or_run *r)
{
    if (!r) return;
    free(r->keys); free(r->pops); free(r->kdiag); free(r->dslot);
    free(r->skeys); free(r->samps); free(r->sinit);
    free(r->dkeys); free(r->kdd); free(r->dsorted); free(r->dsorted_ix); free(r->last_y);
    free(r);
}

/* Excitation level of a determinant relative to D_0: electrons moved. */
static int excit_level(const or_sys *s, const uint64_t *key)
{
    int d = 0;
    for (int x = 0; x < s->W; ++x) d += __builtin_popcountll(key[x] ^ s->ref[x]);
    return d / 2;
}

/* ---- coupled cluster Monte Carlo (Sec. 2.2, eq. ccmc) ----
 * The excitor of determinant D_e moves the electrons of its holes
 * H_e = D_0 \ D_e to its particles P_e = D_e \ D_0. Written as a product of
 * single moves c+_p c_h (k-th lowest hole to k-th lowest particle, applied
 * lowest first), it acts on a determinant D by the second-quantised rules: a
 * move needs h occupied and p empty (else the product vanishes) and gives
 * (-1)^(occupied spin-orbitals strictly between h and p). The excitor a_e is
 * that product times the sign sigma_e making a_e D_0 = +D_e. Pairs c+ c on
 * distinct spin-orbitals commute, so excitors commute and the product of a
 * cluster does not depend on the order of its excitors. */
static int moves_apply(const or_sys *s, const uint64_t *e, uint64_t *D)
{
    int holes[64], parts[64], nh = 0, np = 0;
    for (int P = 0; P < s->n_so; ++P) {
        int in0 = getbit(s->ref, P), ine = getbit(e, P);
        if (in0 && !ine) holes[nh++] = P;
        if (!in0 && ine) parts[np++] = P;
        if (nh == 64 || np == 64) return 0;
    }
    if (nh != np) return 0;
    int sign = 1;
    for (int k = 0; k < nh; ++k) {
        int h = holes[k], p = parts[k];
        if (!getbit(D, h) || getbit(D, p)) return 0;
        if (parity_between(D, h, p) < 0.0) sign = -sign;
        clrbit(D, h);
        setbit(D, p);
    }
    return sign;
}

int or_cluster_collapse(const or_sys *s, const uint64_t *ex, int n, uint64_t *out)
{
    uint64_t D[OR_MAXW], D0[OR_MAXW];
    memcpy(D, s->ref, sizeof(uint64_t) * s->W);
    int sign = 1;
    for (int j = 0; j < n; ++j) {
        const uint64_t *e = ex + (size_t)j * s->W;
        memcpy(D0, s->ref, sizeof(uint64_t) * s->W);
        int sigma = moves_apply(s, e, D0); /* a_e D_0 = sigma * (moves) D_0 = +D_e */
        int m = moves_apply(s, e, D);
        if (sigma == 0 || m == 0) return 0;
        sign *= sigma * m;
    }
    memcpy(out, D, sizeof(uint64_t) * s->W);
    return sign;
}

/* ---- one spawning attempt (Sec. 2.4 "spawning"; Sec. 2.1 real weights) ---- */
static int spawn_attempt(or_run *r, const uint64_t *key, uint64_t h, int32_t n0, int64_t nat, int64_t k,
                         uint8_t init, int parent_in_d)
{
    const or_sys *s = r->s;
    uint32_t w[8], rnd[4];
    uint32_t t = (uint32_t)r->t;
    draw(r, TAG_SELECT, (uint32_t)k, t, h, w);
    draw(r, TAG_SELECT2, (uint32_t)k, t, h, w + 4);
    uint64_t child[OR_MAXW] = {0};
    double pgen = 0.0, hij = 0.0;
    if (!or_exgen(s, r->q.excit_gen, r->q.p_single, key, w, child, &pgen, &hij)) return OR_OK;
    if (hij == 0.0) return OR_OK;
    /* CCMC: amplitudes exist only up to the truncation level */
    if (r->q.method == OR_CCMC && excit_level(s, child) > r->q.ccmc_truncation) return OR_OK;
    if (parent_in_d && dspace_find(r, child) >= 0) return OR_OK;
    double ah = fabs(hij);
    if (r->q.tau_search) {
        double ratio = ah / pgen;
        if (ratio > r->rs_max) r->rs_max = ratio;
    }
    double m;
    if (r->q.fixed_point_bits == 0) {
        m = (r->q.tau * ah) / pgen;
    } else {
        double an = (double)(n0 < 0 ? -(int64_t)n0 : (int64_t)n0);
        m = (((r->q.tau * ah) / pgen) * an) / (double)nat;
    }
    /* the uniform of the stochastic rounding: the Hubbard and electron-gas
       generators use only the first one or two words of the selection block,
       so its last two words serve; heat-bath uses every word and draws a
       block of its own */
    double u;
    if (r->q.excit_gen == OR_EXGEN_HEATBATH) {
        draw(r, TAG_SPAWN_ROUND, (uint32_t)k, t, h, rnd);
        u = u53(rnd[0], rnd[1]);
    } else {
        u = u53(w[2], w[3]);
    }
    if (!(m < 0x1p31)) return OR_EOVERFLOW;
    int64_t kk;
    if (r->q.fixed_point_bits != 0 && m < (double)r->cu)
        kk = (u * (double)r->cu < m) ? r->cu : 0;
    else
        kk = sround(m, u);
    if (kk == 0) return OR_OK;
    if (kk > 2147483647) return OR_EOVERFLOW;
    int sh = hij > 0.0 ? 1 : -1;
    int sn = n0 > 0 ? 1 : -1;
    int32_t amp = (int32_t)(-(sh * sn) * kk);
    push_spawn(r, child, amp, init);
    return OR_OK;
}

/* ---- one spawning attempt of a density-matrix pair (Sec. 2.3) ----
 * DMQMC, eq. (dmqmc): rho_ij gains -(dbeta/2) sum_k [H_ik rho_kj + rho_ik H_kj],
 * so each pair spawns from both ends: attempt a acts on the bra (even a) or
 * the ket (odd a), with the excitation generator of the half it acts on and
 * amplitude (dbeta / 2)|H| / p_gen per walker. IP-DMQMC, eq. (ipdmqmc):
 * df/dtau = H^0 f - f H with H^0 diagonal, so only the ket end spawns, with
 * amplitude dtau |H| / p_gen. The random blocks are those of attempt a of the
 * pair (keyed by the pair's hash). */
static int spawn_attempt_pair(or_run *r, const uint64_t *key, uint64_t h, int32_t n0, int64_t nat, int64_t a,
                              int side)
{
    const or_sys *s = r->s;
    int w = det_words(r);
    uint32_t wv[8], rnd[4];
    uint32_t t = (uint32_t)r->t;
    draw(r, TAG_SELECT, (uint32_t)a, t, h, wv);
    draw(r, TAG_SELECT2, (uint32_t)a, t, h, wv + 4);
    uint64_t half[OR_MAXW] = {0};
    double pgen = 0.0, hij = 0.0;
    if (!or_exgen(s, r->q.excit_gen, r->q.p_single, key + side * w, wv, half, &pgen, &hij)) return OR_OK;
    if (hij == 0.0) return OR_OK;
    uint64_t child[OR_MAXW] = {0};
    memcpy(child, key, sizeof(uint64_t) * r->W);
    memcpy(child + side * w, half, sizeof(uint64_t) * w);
    double ah = fabs(hij);
    double tau = r->q.method == OR_DMQMC ? r->q.tau * 0.5 : r->q.tau;
    double m;
    if (r->q.fixed_point_bits == 0) {
        m = (tau * ah) / pgen;
    } else {
        double an = (double)(n0 < 0 ? -(int64_t)n0 : (int64_t)n0);
        m = (((tau * ah) / pgen) * an) / (double)nat;
    }
    double u;
    if (r->q.excit_gen == OR_EXGEN_HEATBATH) {
        draw(r, TAG_SPAWN_ROUND, (uint32_t)a, t, h, rnd);
        u = u53(rnd[0], rnd[1]);
    } else {
        u = u53(wv[2], wv[3]);
    }
    if (!(m < 0x1p31)) return OR_EOVERFLOW;
    int64_t kk;
    if (r->q.fixed_point_bits != 0 && m < (double)r->cu)
        kk = (u * (double)r->cu < m) ? r->cu : 0;
    else
        kk = sround(m, u);
    if (kk == 0) return OR_OK;
    if (kk > 2147483647) return OR_EOVERFLOW;
    int sh = hij > 0.0 ? 1 : -1;
    int sn = n0 > 0 ? 1 : -1;
    push_spawn(r, child, (int32_t)(-(sh * sn) * kk), 1);
    return OR_OK;
}

/* ---- CCMC: composite clusters (Sec. 2.2: the cluster expansion of t~_j is
 * sampled and each sampled term propagated on its own) ----
 * With T = sum_i N_i a_i over the excitors of the list (not the reference)
 * and t_HF = N_0, Psi = N_0 exp(T / N_0) D_0 expands into terms
 * N_0^(1-s) N_{e_1} ... N_{e_s} a_{e_1} ... a_{e_s} D_0 over sets of s distinct
 * excitors (a repeated excitor gives zero). The terms with s = 0 (D_0) and
 * s = 1 (each excitor on its own determinant) are the list entries
 * themselves and propagate exactly as FCIQMC parents do. Terms with s >= 2
 * are sampled: n_c = ceil(N_ex 2^-b) selections per iteration, N_ex the sum
 * of |N_i| over the excitors. Selection c draws its size s in [2, s_max]
 * with p(s) = 2^-(s-1) (s < s_max) and p(s_max) = 2^-(s_max-2), s_max = the
 * truncation level + 2 (a larger cluster is beyond the reach of H from any
 * amplitude kept), then s excitors independently with probability
 * |N_i| / N_ex each. A set of s distinct excitors is drawn with probability
 * p(s) s! prod |N_i| / N_ex^s, so the term's weight per selection is
 *   w = sgn * N_0 (N_ex / N_0)^s / (p(s) s! n_c)  (units of 2^-b walkers),
 * sgn the sign of N_0^(1-s) prod N_i times the sign of the collapsed
 * product a_{e_1} ... a_{e_s} D_0 = +-D. The term then makes one spawning
 * attempt from D (amplitude dtau |H_jD| w / p_gen, rounded as a parent's) onto
 * a D_j within the truncation level, and, when D itself is within it, the
 * death step of the term, -dtau (K_DD - S) w stochastically rounded, as a
 * spawn onto D. Both are unbiased, so the expected change of each amplitude
 * is -dtau <D_i|K - S|Psi>, eq. (ccmc).
 * Selection order: the excitors ordered by (64-bit hash of the key, key), a
 * cumulative sum of |N_i| in that order, and a 64-bit uniform integer r
 * mapped to floor(r N_ex / 2^64) within it. Random numbers: Philox under the
 * key (seed_lo, seed_hi ^ replica_id ^ 2^31), counter (tag, draw, t, c). */
static void draw_cluster(const or_run *r, uint32_t tag, uint32_t k, uint32_t t, uint64_t c, uint32_t out[4])
{
    uint32_t ctr[4] = {(tag << 28) | k, t, (uint32_t)c, (uint32_t)(c >> 32)};
    uint32_t key[2] = {r->rkey[0], r->rkey[1] ^ 0x80000000u};
    or_philox4x32_10(ctr, key, out);
}

static struct { const or_run *r; const uint64_t *h; } g_hord;
static int hash_order_cmp(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t hi = g_hord.h[i], hj = g_hord.h[j];
    if (hi != hj) return hi < hj ? -1 : 1;
    return key_cmp(g_hord.r->keys + (size_t)i * g_hord.r->W, g_hord.r->keys + (size_t)j * g_hord.r->W, g_hord.r->W);
}

/* one spawning attempt of a sampled cluster (collapsed determinant D,
   weight magnitude mag and sign sw); random blocks as an attempt 0 of a
   parent with hash c, under the cluster key */
static int cluster_spawn(or_run *r, const uint64_t *D, uint64_t c, double mag, int sw)
{
    const or_sys *s = r->s;
    uint32_t w[8], rnd[4];
    uint32_t t = (uint32_t)r->t;
    draw_cluster(r, TAG_SELECT, 0, t, c, w);
    draw_cluster(r, TAG_SELECT2, 0, t, c, w + 4);
    uint64_t child[OR_MAXW] = {0};
    double pgen = 0.0, hij = 0.0;
    if (!or_exgen(s, r->q.excit_gen, r->q.p_single, D, w, child, &pgen, &hij)) return OR_OK;
    if (hij == 0.0) return OR_OK;
    if (excit_level(s, child) > r->q.ccmc_truncation) return OR_OK;
    double ah = fabs(hij);
    double m = ((r->q.tau * ah) / pgen) * mag;
    double u;
    if (r->q.excit_gen == OR_EXGEN_HEATBATH) {
        draw_cluster(r, TAG_SPAWN_ROUND, 0, t, c, rnd);
        u = u53(rnd[0], rnd[1]);
    } else {
        u = u53(w[2], w[3]);
    }
    if (!(m < 0x1p31)) return OR_EOVERFLOW;
    int64_t kk;
    if (r->q.fixed_point_bits != 0 && m < (double)r->cu)
        kk = (u * (double)r->cu < m) ? r->cu : 0;
    else
        kk = sround(m, u);
    if (kk == 0) return OR_OK;
    if (kk > 2147483647) return OR_EOVERFLOW;
    int sh = hij > 0.0 ? 1 : -1;
    push_spawn(r, child, (int32_t)(-(sh * sw) * kk), 1);
    return OR_OK;
}

static int ccmc_composite(or_run *r, int32_t n0)
{
    const or_sys *s = r->s;
    int W = r->W;
    uint32_t t = (uint32_t)r->t;
    int trunc = r->q.ccmc_truncation;
    int smax = trunc + 2 < s->nel ? trunc + 2 : s->nel;
    /* the excitors in (hash, key) order and the cumulative sum of |N_i| */
    int64_t ne = 0;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(r->n ? r->n : 1));
    uint64_t *hh = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(r->n ? r->n : 1));
    for (int64_t i = 0; i < r->n; ++i) {
        hh[i] = or_hash64(r->keys + (size_t)i * W, W);
        if (!is_reference(r, r->keys + (size_t)i * W)) ord[ne++] = i;
    }
    g_hord.r = r;
    g_hord.h = hh;
    qsort(ord, (size_t)ne, sizeof(int64_t), hash_order_cmp);
    int64_t *cum = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ne + 1));
    cum[0] = 0;
    for (int64_t x = 0; x < ne; ++x) {
        int32_t p = r->pops[ord[x]];
        cum[x + 1] = cum[x] + (p < 0 ? -(int64_t)p : p);
    }
    int64_t nex = cum[ne];
    int b = r->q.fixed_point_bits;
    int64_t nc = b ? (nex + ((int64_t)1 << b) - 1) >> b : nex;
    int status = OR_OK;
    double an0 = (double)(n0 < 0 ? -(int64_t)n0 : (int64_t)n0);
    for (int64_t c = 0; c < nc && smax >= 2 && status == OR_OK; ++c) {
        uint32_t rr[4];
        draw_cluster(r, TAG_CLUSTER, 0, t, (uint64_t)c, rr);
        double u = u53(rr[0], rr[1]);
        int sz = 2;
        while (sz < smax && u >= 1.0 - ldexp(1.0, -(sz - 1))) ++sz;
        double ps = sz < smax ? ldexp(1.0, -(sz - 1)) : ldexp(1.0, -(smax - 2));
        int64_t pick_ix[8];
        uint64_t ex[8 * OR_MAXW];
        int sgn = 1, dup = 0;
        for (int j = 0; j < sz; ++j) {
            draw_cluster(r, TAG_CLUSTER, (uint32_t)(1 + j), t, (uint64_t)c, rr);
            uint64_t r64 = ((uint64_t)rr[0] << 32) | rr[1];
            int64_t target = (int64_t)(((unsigned __int128)r64 * (uint64_t)nex) >> 64);
            int64_t lo = 0, hi = ne; /* last x with cum[x] <= target */
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) / 2;
                if (cum[mid] <= target) lo = mid; else hi = mid;
            }
            pick_ix[j] = ord[lo];
            for (int q = 0; q < j; ++q) dup |= pick_ix[q] == pick_ix[j];
            memcpy(ex + (size_t)j * W, r->keys + (size_t)pick_ix[j] * W, sizeof(uint64_t) * W);
            if (r->pops[pick_ix[j]] < 0) sgn = -sgn;
        }
        if (dup) continue;
        uint64_t D[OR_MAXW];
        int cs = or_cluster_collapse(s, ex, sz, D);
        if (cs == 0) continue;
        int lev = excit_level(s, D);
        if (lev > trunc + 2) continue;
        sgn *= cs;
        if ((sz % 2 == 0) && n0 < 0) sgn = -sgn; /* sign of N_0^(1-s) */
        double x = (double)nex / an0;
        double f = x;
        for (int j = 1; j < sz; ++j) f = f * x;
        double fact = 1.0;
        for (int j = 2; j <= sz; ++j) fact *= (double)j;
        double mag = (an0 * f) / ((ps * fact) * (double)nc);
        status = cluster_spawn(r, D, (uint64_t)c, mag, sgn);
        if (status != OR_OK || lev > trunc) continue;
        /* the death step of the term, as a spawn onto D */
        double md = (r->q.tau * ((or_diag(s, D) - s->H00) - r->S)) * mag;
        draw_cluster(r, TAG_DEATH, 0, t, (uint64_t)c, rr);
        double ud = u53(rr[0], rr[1]);
        if (!(fabs(md) < 0x1p31)) { status = OR_EOVERFLOW; break; }
        int64_t k = sround(fabs(md), ud);
        if (k == 0) continue;
        int dsg = md >= 0.0 ? -sgn : sgn;
        push_spawn(r, D, (int32_t)(dsg * k), 1);
    }
    free(ord); free(hh); free(cum);
    return status;
}

typedef struct { const uint64_t *keys; int W; } sort_ctx_t;
static sort_ctx_t g_sort;
static int idx_cmp(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    int c = key_cmp(g_sort.keys + (size_t)i * g_sort.W, g_sort.keys + (size_t)j * g_sort.W, g_sort.W);
    if (c) return c;
    return (i > j) - (i < j);
}

/* Deterministic projection on D (Sec. 2.1 semi-stochastic propagation):
 * y_i = sum_j K_ij n_j. Reading: the sum is taken exactly and rounded once,
 * as the projected-energy numerator is: every FP64 product K_ij n_j is
 * truncated at 2^-64 and added in fixed point, so the value does not depend
 * on the order of the terms. */
static double det_row(const double *row, const double *c, int64_t nd)
{
    int64_t limbs[4] = {0, 0, 0, 0};
    for (int64_t j = 0; j < nd; ++j) acc_term(limbs, row[j] * c[j]);
    return limbs_value(limbs);
}

static struct { const or_run *r; } g_top;
static int top_cmp(const void *a, const void *b)
{
    const or_run *r = g_top.r;
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    int64_t ai = r->pops[i] < 0 ? -(int64_t)r->pops[i] : r->pops[i];
    int64_t aj = r->pops[j] < 0 ? -(int64_t)r->pops[j] : r->pops[j];
    if (ai != aj) return ai > aj ? -1 : 1;
    return key_cmp(r->keys + (size_t)i * r->W, r->keys + (size_t)j * r->W, r->W);
}

/* D given as nd keys in D order: mark the entries, build K_DD and the sorted
   copy used for membership tests. Every key must be in the list. */
static void install_detspace(or_run *r, const uint64_t *dkeys, int64_t nd)
{
    int W = r->W;
    r->nd = nd;
    r->dkeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nd ? nd : 1) * W);
    r->kdd = (double *)malloc(sizeof(double) * (size_t)(nd ? nd * nd : 1));
    r->last_y = (double *)calloc((size_t)(nd ? nd : 1), sizeof(double));
    memcpy(r->dkeys, dkeys, sizeof(uint64_t) * (size_t)nd * W);
    int64_t *at = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd ? nd : 1));
    for (int64_t d = 0; d < nd; ++d) {
        /* the list is sorted by key */
        int64_t lo = 0, hi = r->n;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (key_cmp(r->keys + (size_t)mid * W, dkeys + (size_t)d * W, W) < 0) lo = mid + 1; else hi = mid;
        }
        at[d] = lo;
        r->dslot[lo] = (int32_t)d;
    }
    for (int64_t d = 0; d < nd; ++d)
        for (int64_t e = 0; e < nd; ++e) {
            double v;
            if (d == e)
                v = r->kdiag[at[d]];
            else
                v = or_hij(r->s, r->dkeys + (size_t)d * W, r->dkeys + (size_t)e * W);
            r->kdd[d * nd + e] = v;
        }
    free(at);
    /* sorted copy for membership tests */
    g_sort.keys = r->dkeys;
    g_sort.W = W;
    int64_t *sx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd ? nd : 1));
    for (int64_t d = 0; d < nd; ++d) sx[d] = d;
    qsort(sx, (size_t)nd, sizeof(int64_t), idx_cmp);
    r->dsorted = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nd ? nd : 1) * W);
    r->dsorted_ix = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nd ? nd : 1));
    for (int64_t d = 0; d < nd; ++d) {
        memcpy(r->dsorted + (size_t)d * W, r->dkeys + (size_t)sx[d] * W, sizeof(uint64_t) * W);
        r->dsorted_ix[d] = (int32_t)sx[d];
    }
    free(sx);
    r->ss_active = 1;
}

static void select_detspace(or_run *r)
{
    int64_t nd = r->q.ss_size < r->n ? r->q.ss_size : r->n;
    /* order: |n| descending, then key ascending (a total order: keys are distinct) */
    int64_t *ix = (int64_t *)malloc(sizeof(int64_t) * (size_t)(r->n ? r->n : 1));
    for (int64_t i = 0; i < r->n; ++i) ix[i] = i;
    g_top.r = r;
    qsort(ix, (size_t)r->n, sizeof(int64_t), top_cmp);
    uint64_t *dk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nd ? nd : 1) * r->W);
    for (int64_t d = 0; d < nd; ++d) memcpy(dk + (size_t)d * r->W, r->keys + (size_t)ix[d] * r->W, sizeof(uint64_t) * r->W);
    free(ix);
    install_detspace(r, dk, nd);
    free(dk);
}

/* ---- one deterministic space shared by several runs of one system ---- */
typedef struct { const uint64_t *key; int64_t sum; } tot_t;
static int g_tot_w;
static int tot_key_cmp(const void *a, const void *b)
{
    return key_cmp(((const tot_t *)a)->key, ((const tot_t *)b)->key, g_tot_w);
}
static int tot_rank_cmp(const void *a, const void *b)
{
    const tot_t *x = (const tot_t *)a, *y = (const tot_t *)b;
    if (x->sum != y->sum) return x->sum > y->sum ? -1 : 1;
    return key_cmp(x->key, y->key, g_tot_w);
}

/* insert the given keys (sorted, absent from the list) with n = 0 */
static void insert_zero_entries(or_run *r, const uint64_t *add, int64_t na)
{
    int W = r->W;
    int64_t n = r->n, tot = n + na;
    uint64_t *nk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(tot ? tot : 1) * W);
    int32_t *np = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    double *nkd = (double *)malloc(sizeof(double) * (size_t)(tot ? tot : 1));
    int32_t *nds = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    int64_t i = 0, j = 0, o = 0;
    while (i < n || j < na) {
        int take_old = j >= na || (i < n && key_cmp(r->keys + (size_t)i * W, add + (size_t)j * W, W) < 0);
        if (take_old) {
            memcpy(nk + (size_t)o * W, r->keys + (size_t)i * W, sizeof(uint64_t) * W);
            np[o] = r->pops[i];
            nkd[o] = r->kdiag[i];
            nds[o] = r->dslot[i];
            ++i;
        } else {
            memcpy(nk + (size_t)o * W, add + (size_t)j * W, sizeof(uint64_t) * W);
            np[o] = 0;
            nkd[o] = entry_kdiag(r, add + (size_t)j * W);
            nds[o] = -1;
            ++j;
        }
        ++o;
    }
    free(r->keys); free(r->pops); free(r->kdiag); free(r->dslot);
    r->keys = nk; r->pops = np; r->kdiag = nkd; r->dslot = nds;
    r->n = tot;
    r->cap = tot;
}

int or_runs_select_shared(or_run **runs, int nr)
{
    if (nr <= 0) return OR_EINVAL;
    int W = runs[0]->W;
    int64_t size = runs[0]->q.ss_size, total = 0;
    for (int k = 0; k < nr; ++k) total += runs[k]->n;
    /* summed |n| over the runs of every occupied determinant */
    tot_t *all = (tot_t *)malloc(sizeof(tot_t) * (size_t)(total ? total : 1));
    int64_t m = 0;
    for (int k = 0; k < nr; ++k)
        for (int64_t i = 0; i < runs[k]->n; ++i) {
            all[m].key = runs[k]->keys + (size_t)i * W;
            all[m].sum = runs[k]->pops[i] < 0 ? -(int64_t)runs[k]->pops[i] : runs[k]->pops[i];
            ++m;
        }
    g_tot_w = W;
    qsort(all, (size_t)m, sizeof(tot_t), tot_key_cmp);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (u > 0 && key_cmp(all[u - 1].key, all[i].key, W) == 0)
            all[u - 1].sum += all[i].sum;
        else
            all[u++] = all[i];
    }
    if (u < size) { free(all); return OR_EINVAL; }
    qsort(all, (size_t)u, sizeof(tot_t), tot_rank_cmp);
    uint64_t *dk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(size ? size : 1) * W);
    for (int64_t d = 0; d < size; ++d) memcpy(dk + (size_t)d * W, all[d].key, sizeof(uint64_t) * W);
    free(all);
    /* sorted copy of D, for the members a run does not hold */
    int64_t *sx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(size ? size : 1));
    for (int64_t d = 0; d < size; ++d) sx[d] = d;
    g_sort.keys = dk;
    g_sort.W = W;
    qsort(sx, (size_t)size, sizeof(int64_t), idx_cmp);
    uint64_t *add = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(size ? size : 1) * W);
    for (int k = 0; k < nr; ++k) {
        or_run *r = runs[k];
        int64_t na = 0;
        for (int64_t x = 0; x < size; ++x) {
            const uint64_t *key = dk + (size_t)sx[x] * W;
            int64_t lo = 0, hi = r->n;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (key_cmp(r->keys + (size_t)mid * W, key, W) < 0) lo = mid + 1; else hi = mid;
            }
            if (lo == r->n || key_cmp(r->keys + (size_t)lo * W, key, W) != 0)
                memcpy(add + (size_t)(na++) * W, key, sizeof(uint64_t) * W);
        }
        if (na) insert_zero_entries(r, add, na);
        install_detspace(r, dk, size);
    }
    free(add);
    free(sx);
    free(dk);
    return OR_OK;
}

static int step_once(or_run *r)
{
    const or_sys *s = r->s;
    int W = r->W;
    r->t += 1;
    uint32_t t = (uint32_t)r->t;
    int64_t n = r->n;
    int64_t flips = 0;
    /* CCMC: the cluster weights divide by t_HF = N_0 */
    int32_t ccmc_n0 = 0;
    if (r->q.method == OR_CCMC) {
        for (int64_t i = 0; i < n; ++i)
            if (is_reference(r, r->keys + (size_t)i * W)) ccmc_n0 = r->pops[i];
        if (ccmc_n0 == 0) return OR_ENOREF;
    }
    /* 1. spawning from the start-of-iteration populations */
    r->ns = 0;
    r->kd_any = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t n0 = r->pops[i];
        if (n0 == 0) continue;
        const uint64_t *key = r->keys + (size_t)i * W;
        if (r->q.fixed_point_bits == 0 && (n0 >= (1 << 28) || n0 <= -(1 << 28))) return OR_EOVERFLOW;
        uint64_t h = or_hash64(key, W);
        int64_t nat = n_attempts(r, n0);
        if (r->q.method == OR_DMQMC) {
            /* nat attempts at each end: attempt 2k acts on the bra, 2k + 1 on the ket */
            if (2 * nat >= ((int64_t)1 << 28)) return OR_EOVERFLOW;
            for (int64_t k = 0; k < nat; ++k)
                for (int side = 0; side < 2; ++side) {
                    int st = spawn_attempt_pair(r, key, h, n0, nat, 2 * k + side, side);
                    if (st) return st;
                }
            continue;
        }
        if (r->q.method == OR_IPDMQMC) {
            for (int64_t k = 0; k < nat; ++k) {
                int st = spawn_attempt_pair(r, key, h, n0, nat, k, 1);
                if (st) return st;
            }
            continue;
        }
        int64_t an = n0 < 0 ? -(int64_t)n0 : n0;
        int pin_d = r->ss_active && r->dslot[i] >= 0;
        uint8_t init = (uint8_t)(an > r->thr || is_reference(r, key) || pin_d);
        for (int64_t k = 0; k < nat; ++k) {
            int st = spawn_attempt(r, key, h, n0, nat, k, init, pin_d);
            if (st) return st;
        }
    }
    int64_t n_cluster = r->ns;
    if (r->q.method == OR_CCMC) {
        int st = ccmc_composite(r, ccmc_n0);
        if (st) return st;
    }
    n_cluster = r->ns - n_cluster;
    /* 2. death/cloning (Sec. 2.4 "death"; shift as diagonal offset, Sec. 2.1),
     *    3. deterministic projection for D entries; both from start-of-iteration values */
    int64_t *newpop = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    double *cvec = NULL;
    if (r->ss_active) {
        cvec = (double *)calloc((size_t)(r->nd ? r->nd : 1), sizeof(double));
        for (int64_t i = 0; i < n; ++i)
            if (r->dslot[i] >= 0) cvec[r->dslot[i]] = (double)r->pops[i];
        for (int64_t d = 0; d < r->nd; ++d) r->last_y[d] = det_row(r->kdd + d * r->nd, cvec, r->nd);
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t n0 = r->pops[i];
        const uint64_t *key = r->keys + (size_t)i * W;
        uint64_t h = or_hash64(key, W);
        uint32_t rnd[4];
        if (r->ss_active && r->dslot[i] >= 0) {
            int64_t d = r->dslot[i];
            double delta = (-r->q.tau) * (r->last_y[d] - r->S * (double)n0);
            draw(r, TAG_SEMISTOCH, 0, t, h, rnd);
            double u = u53(rnd[0], rnd[1]);
            if (!(fabs(delta) < 0x1p40)) { free(newpop); free(cvec); return OR_EOVERFLOW; }
            int64_t k = delta >= 0.0 ? sround(delta, u) : -sround(-delta, u);
            newpop[i] = (int64_t)n0 + k;
            continue;
        }
        if (n0 == 0) { newpop[i] = 0; continue; }
        if (r->q.tau_search && (!r->kd_any || r->kdiag[i] > r->kd_max)) {
            r->kd_max = r->kdiag[i];
            r->kd_any = 1;
        }
        double an = (double)(n0 < 0 ? -(int64_t)n0 : (int64_t)n0);
        double m = (r->q.tau * (r->kdiag[i] - r->S)) * an;
        draw(r, TAG_DEATH, 0, t, h, rnd);
        double u = u53(rnd[0], rnd[1]);
        if (!(fabs(m) < 0x1p40)) { free(newpop); free(cvec); return OR_EOVERFLOW; }
        int64_t k = m >= 0.0 ? sround(m, u) : -sround(-m, u);
        int64_t sg = n0 > 0 ? 1 : -1;
        int64_t v = (int64_t)n0 - sg * k;
        if ((v > 0 && n0 < 0) || (v < 0 && n0 > 0)) ++flips;
        newpop[i] = v;
    }
    free(cvec);
    /* 4. annihilation (Sec. 2.4; appendix "Parallelization"): sort the spawned
     *    walkers, combine those on the same determinant, merge into the main list */
    int64_t ns = r->ns;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) ord[i] = i;
    g_sort.keys = r->skeys;
    g_sort.W = W;
    qsort(ord, (size_t)ns, sizeof(int64_t), idx_cmp);
    int64_t nu = 0;
    uint64_t *ukeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(ns > 0 ? ns : 1) * W);
    int64_t *usum = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    uint8_t *uflag = (uint8_t *)malloc((size_t)(ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) {
        const uint64_t *k = r->skeys + (size_t)ord[i] * W;
        if (nu > 0 && key_cmp(ukeys + (size_t)(nu - 1) * W, k, W) == 0) {
            usum[nu - 1] += r->samps[ord[i]];
            uflag[nu - 1] |= r->sinit[ord[i]];
        } else {
            memcpy(ukeys + (size_t)nu * W, k, sizeof(uint64_t) * W);
            usum[nu] = r->samps[ord[i]];
            uflag[nu] = r->sinit[ord[i]];
            ++nu;
        }
    }
    free(ord);
    int64_t cap2 = n + nu + 1;
    uint64_t *nk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cap2 * W);
    int32_t *np = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap2);
    double *nkd = (double *)malloc(sizeof(double) * (size_t)cap2);
    int32_t *nds = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap2);
    int64_t a = 0, b = 0, o = 0, rejected = 0, rejected_sum = 0, death_sum = 0, spawn_sum = 0;
    for (int64_t i = 0; i < n; ++i) death_sum += newpop[i];
    for (int64_t i = 0; i < ns; ++i) spawn_sum += r->samps[i];
    int status = OR_OK;
    while (a < n || b < nu) {
        int c;
        if (a >= n) c = 1;
        else if (b >= nu) c = -1;
        else c = key_cmp(r->keys + (size_t)a * W, ukeys + (size_t)b * W, W);
        int64_t v;
        if (c <= 0) {
            v = newpop[a];
            if (c == 0) { v += usum[b]; ++b; }
            if (v > 2147483647 || v < -2147483647) status = OR_EOVERFLOW;
            if (v != 0 || r->dslot[a] >= 0) {
                memcpy(nk + (size_t)o * W, r->keys + (size_t)a * W, sizeof(uint64_t) * W);
                np[o] = (int32_t)v;
                nkd[o] = r->kdiag[a];
                nds[o] = r->dslot[a];
                ++o;
            }
            ++a;
        } else {
            /* initiator rule (Sec. 2.1): a new determinant only from an initiator parent */
            v = usum[b];
            int accept = (!r->q.initiator || uflag[b]) && v != 0;
            if (accept) {
                if (v > 2147483647 || v < -2147483647) status = OR_EOVERFLOW;
                memcpy(nk + (size_t)o * W, ukeys + (size_t)b * W, sizeof(uint64_t) * W);
                np[o] = (int32_t)v;
                nkd[o] = entry_kdiag(r, ukeys + (size_t)b * W);
                nds[o] = -1;
                ++o;
            } else {
                rejected += v < 0 ? -v : v;
                rejected_sum += v;
            }
            ++b;
        }
    }
    free(newpop); free(ukeys); free(usum); free(uflag);
    if (status != OR_OK) { free(nk); free(np); free(nkd); free(nds); return status; }
    free(r->keys); free(r->pops); free(r->kdiag); free(r->dslot);
    r->keys = nk; r->pops = np; r->kdiag = nkd; r->dslot = nds;
    r->n = o;
    r->cap = cap2;
    /* 5. estimators on the new list */
    compute_estimators(r);
    r->est.n_spawned = ns;
    r->est.n_cluster_spawns = n_cluster;
    r->est.n_sign_flips = flips;
    r->est.n_rejected_units = rejected;
    r->est.n_spawn_events = nu;
    r->est.death_sum = death_sum;
    r->est.spawn_sum = spawn_sum;
    r->est.rejected_sum = rejected_sum;
    /* 6. shift update every A iterations (Sec. 2.1: diagonal energy offset) */
    if (r->t % r->q.shift_period == 0) {
        int64_t nw = r->est.n_walkers_units;
        double target = r->q.target_population * ldexp(1.0, r->q.fixed_point_bits);
        if (!r->vary) {
            if ((double)nw >= target) { r->vary = 1; r->nprev = nw; }
        } else {
            double c = r->q.shift_damping / ((double)r->q.shift_period * r->q.tau);
            double ratio = (double)nw / (double)r->nprev;
            r->S = r->S - c * log(ratio);
            r->nprev = nw;
        }
        r->est.shift = r->S;
        r->est.vary_shift = r->vary;
        /* time-step search (reading of the tutorial's tau_search): after the
           shift update, tau only decreases, to the largest value at which no
           attempt seen so far expects more than one walker per parent walker
           (tau |H_ji| / p_gen <= 1) and the death step of the last iteration
           removes at most every walker of a determinant (tau (K_ii - S) <= 1) */
        if (r->q.tau_search) {
            double tau = r->q.tau;
            if (r->rs_max > 0.0) {
                double b = 1.0 / r->rs_max;
                if (b < tau) tau = b;
            }
            if (r->kd_any) {
                double d = r->kd_max - r->S;
                if (d > 0.0) {
                    double b = 1.0 / d;
                    if (b < tau) tau = b;
                }
            }
            r->q.tau = tau;
        }
    }
    r->est.tau = r->q.tau;
    r->est.spawn_ratio_max = r->rs_max;
    /* deterministic space chosen from the most highly weighted determinants */
    if (r->q.ss_size > 0 && !r->q.ss_shared && !r->ss_active && r->t >= r->q.ss_start_iteration) select_detspace(r);
    return OR_OK;
}

int or_run_step(or_run *r, int n_iter)
{
    for (int i = 0; i < n_iter; ++i) {
        int st = step_once(r);
        if (st) { r->est.status = st; return st; }
    }
    return OR_OK;
}

void or_run_estimators(const or_run *r, or_estimators *out) { *out = r->est; }
int64_t or_run_size(const or_run *r) { return r->n; }

void or_run_export(const or_run *r, uint64_t *keys, int32_t *pops)
{
    memcpy(keys, r->keys, sizeof(uint64_t) * (size_t)r->n * r->W);
    memcpy(pops, r->pops, sizeof(int32_t) * (size_t)r->n);
}

int or_run_import(or_run *r, const uint64_t *keys, const int32_t *pops, int64_t n, double shift,
                  int64_t iteration, int32_t vary, int64_t n_prev)
{
    int W = r->W;
    int64_t *ix = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) ix[i] = i;
    g_sort.keys = keys;
    g_sort.W = W;
    qsort(ix, (size_t)n, sizeof(int64_t), idx_cmp);
    for (int64_t i = 1; i < n; ++i)
        if (key_cmp(keys + (size_t)ix[i] * W, keys + (size_t)ix[i - 1] * W, W) == 0) {
            free(ix);
            return OR_EINVAL;
        }
    /* CCMC: no amplitude beyond the truncation level */
    for (int64_t i = 0; i < n && r->q.method == OR_CCMC; ++i)
        if (excit_level(r->s, keys + (size_t)i * W) > r->q.ccmc_truncation) {
            free(ix);
            return OR_EINVAL;
        }
    free(r->keys); free(r->pops); free(r->kdiag); free(r->dslot);
    r->keys = NULL; r->pops = NULL; r->kdiag = NULL; r->dslot = NULL; r->cap = 0;
    list_reserve(r, n ? n : 1);
    int64_t o = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (pops[ix[i]] == 0) continue;
        memcpy(r->keys + (size_t)o * W, keys + (size_t)ix[i] * W, sizeof(uint64_t) * W);
        r->pops[o] = pops[ix[i]];
        r->kdiag[o] = entry_kdiag(r, keys + (size_t)ix[i] * W);
        r->dslot[o] = -1;
        ++o;
    }
    free(ix);
    r->n = o;
    r->S = shift;
    r->t = iteration;
    r->vary = vary;
    r->nprev = n_prev;
    free(r->dkeys); free(r->kdd); free(r->dsorted); free(r->dsorted_ix); free(r->last_y);
    r->dkeys = NULL; r->kdd = NULL; r->dsorted = NULL; r->dsorted_ix = NULL; r->last_y = NULL;
    r->ss_active = 0;
    r->nd = 0;
    compute_estimators(r);
    if (r->q.ss_size > 0 && !r->q.ss_shared && r->t >= r->q.ss_start_iteration) select_detspace(r);
    return OR_OK;
}

int64_t or_run_n_spawns(const or_run *r) { return r->ns; }

void or_run_spawns(const or_run *r, uint64_t *keys, int32_t *amps, uint8_t *init)
{
    memcpy(keys, r->skeys, sizeof(uint64_t) * (size_t)r->ns * r->W);
    memcpy(amps, r->samps, sizeof(int32_t) * (size_t)r->ns);
    memcpy(init, r->sinit, (size_t)r->ns);
}

int64_t or_run_detspace(const or_run *r, uint64_t *keys)
{
    if (keys && r->nd) memcpy(keys, r->dkeys, sizeof(uint64_t) * (size_t)r->nd * r->W);
    return r->nd;
}

void or_run_last_projection(const or_run *r, double *y)
{
    if (r->nd) memcpy(y, r->last_y, sizeof(double) * (size_t)r->nd);
}
