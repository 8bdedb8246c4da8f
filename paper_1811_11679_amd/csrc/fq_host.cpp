// Host half of the FCIQMC library: the C ABI of include/fciqmc.h.
//
// Builds the per-system device tables (UEG plane-wave basis, kinetic and
// Coulomb tables, momentum grid; molecular integrals and heat-bath tables),
// carves the caller's workspace into the main lists, the spawned list and the
// sort/merge scratch, enqueues iterations on the caller's stream and runs the
// shift update of the paper (Sec. 2.1: diagonal energy offset; tutorial
// appendix: mc_cycles, target_population) on the host between iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fciqmc.h"
#include "fq_kernels.h"

using namespace fq;

namespace {

constexpr int HIST_LEN = 128;
constexpr uint64_t HOST_HASH_SEED = 0x9E3779B97F4A7C15ull;

// MurmurHash64A over the key words (host copy of the device definition)
uint64_t host_hash(const uint64_t *k, int W)
{
    const uint64_t m = 0xc6a4a7935bd1e995ull;
    uint64_t h = HOST_HASH_SEED ^ ((uint64_t)(8 * W) * m);
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

uint64_t host_skey(uint64_t h, uint32_t rep, int rb) { return rb ? (((uint64_t)rep << (64 - rb)) | (h >> rb)) : h; }

int key_cmp_host(const uint64_t *a, const uint64_t *b, int W)
{
    for (int i = W - 1; i >= 0; --i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

int round_w(int n_so)
{
    const int w = (n_so + 63) / 64;
    if (w <= 1) return 1;
    if (w <= 2) return 2;
    if (w <= 4) return 4;
    return 8;
}

// Host description of one system and the tables it ships to the device.
struct HostSys {
    int kind = 0, n_spatial = 0, n_so = 0, nel = 0, na = 0, nb = 0, periodic = 0;
    double t = 0, U = 0, L = 0, k2 = 0, vc = 0;
    int gmax = 0, gdim = 0, vlen = 0;
    std::vector<int32_t> npk;
    std::vector<double> eps, vtab, vx;
    std::vector<int16_t> grid;
    std::vector<double> h1, eri, hd, Jt, Kt;
    std::vector<int64_t> hb_off;
    std::vector<int32_t> hb_cnt;
    std::vector<double> hb_S, hb_cdf;
    std::vector<uint16_t> hb_AB;
    uint64_t ref[MAXW] = {0};
};

void setbit_h(uint64_t *k, int P) { k[P >> 6] |= 1ull << (P & 63); }

double antisym_mol(const HostSys &s, int A, int B, int P, int Q)
{
    const int n = s.n_spatial;
    auto e = [&](int p, int q, int r, int t) { return s.eri[(((size_t)p * n + q) * n + r) * n + t]; };
    const int sa = A & 1, sb = B & 1, sp = P & 1, sq = Q & 1;
    const double x = (sa == sp && sb == sq) ? e(A >> 1, P >> 1, B >> 1, Q >> 1) : 0.0;
    const double y = (sa == sq && sb == sp) ? e(A >> 1, Q >> 1, B >> 1, P >> 1) : 0.0;
    return x - y;
}

std::string build_system(const fq_system &d, HostSys &s)
{
    s.kind = d.kind;
    s.na = d.n_alpha;
    s.nb = d.n_beta;
    s.nel = d.n_alpha + d.n_beta;
    if (d.n_alpha < 0 || d.n_beta < 0 || s.nel < 2) return "need at least two electrons";
    if (d.kind == FQ_HUBBARD_REAL) {
        if (d.n_sites < 3 || d.n_sites > 32) return "Hubbard chain needs 3..32 sites";
        if (d.n_alpha > d.n_sites || d.n_beta > d.n_sites) return "too many electrons for the chain";
        s.n_spatial = d.n_sites;
        s.periodic = d.periodic ? 1 : 0;
        s.t = d.t;
        s.U = d.U;
        int placed = 0;
        for (int pass = 0; pass < 2 && placed < d.n_alpha; ++pass)
            for (int p = pass; p < d.n_sites && placed < d.n_alpha; p += 2, ++placed) setbit_h(s.ref, 2 * p);
        placed = 0;
        for (int pass = 1; pass >= 0 && placed < d.n_beta; --pass)
            for (int p = pass; p < d.n_sites && placed < d.n_beta; p += 2, ++placed) setbit_h(s.ref, 2 * p + 1);
    } else if (d.kind == FQ_UEG) {
        if (d.ecut_n2 < 1 || !(d.rs > 0)) return "UEG needs rs > 0 and ecut_n2 >= 1";
        int c = 0;
        while ((c + 1) * (c + 1) <= d.ecut_n2) ++c;
        struct PW { int n2, x, y, z; };
        std::vector<PW> pw;
        for (int x = -c; x <= c; ++x)
            for (int y = -c; y <= c; ++y)
                for (int z = -c; z <= c; ++z) {
                    const int n2 = x * x + y * y + z * z;
                    if (n2 <= d.ecut_n2) pw.push_back({n2, x, y, z});
                }
        std::sort(pw.begin(), pw.end(), [](const PW &a, const PW &b) {
            if (a.n2 != b.n2) return a.n2 < b.n2;
            if (a.x != b.x) return a.x < b.x;
            if (a.y != b.y) return a.y < b.y;
            return a.z < b.z;
        });
        const int M = (int)pw.size();
        if (2 * M > 64 * MAXW) return "UEG basis exceeds 512 spin-orbitals";
        if (d.n_alpha > M || d.n_beta > M) return "too many electrons for the basis";
        s.n_spatial = M;
        s.npk.resize(M);
        s.eps.resize(M);
        for (int i = 0; i < M; ++i)
            s.npk[i] = (pw[i].x + 256) | ((pw[i].y + 256) << 10) | ((pw[i].z + 256) << 20);
        const double N = (double)s.nel;
        s.L = d.rs * std::cbrt((4.0 * M_PI * N) / 3.0);
        const double g = (2.0 * M_PI) / s.L;
        s.k2 = g * g;
        s.vc = (4.0 * M_PI) / ((s.L * s.L) * s.L);
        for (int i = 0; i < M; ++i) s.eps[i] = (s.k2 * (double)pw[i].n2) * 0.5;
        s.vlen = 4 * d.ecut_n2 + 1;
        s.vtab.assign(s.vlen, 0.0);
        for (int q = 1; q < s.vlen; ++q) s.vtab[q] = s.vc / (s.k2 * (double)q);
        s.vx.assign((size_t)M * M, 0.0);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                const int dx = pw[i].x - pw[j].x, dy = pw[i].y - pw[j].y, dz = pw[i].z - pw[j].z;
                s.vx[(size_t)i * M + j] = s.vtab[dx * dx + dy * dy + dz * dz];
            }
        s.gmax = 3 * c;
        s.gdim = 2 * s.gmax + 1;
        s.grid.assign((size_t)s.gdim * s.gdim * s.gdim, (int16_t)-1);
        for (int i = 0; i < M; ++i)
            s.grid[((size_t)(pw[i].x + s.gmax) * s.gdim + (pw[i].y + s.gmax)) * s.gdim + (pw[i].z + s.gmax)] =
                (int16_t)i;
        for (int i = 0; i < d.n_alpha; ++i) setbit_h(s.ref, 2 * i);
        for (int i = 0; i < d.n_beta; ++i) setbit_h(s.ref, 2 * i + 1);
    } else if (d.kind == FQ_MOLECULAR) {
        const int n = d.n_orb;
        if (n <= 0 || 2 * n > 128 || !d.h1 || !d.eri) return "molecular system needs 1..64 orbitals and integrals";
        if (d.n_alpha > n || d.n_beta > n) return "too many electrons for the orbitals";
        s.n_spatial = n;
        s.h1.assign(d.h1, d.h1 + (size_t)n * n);
        s.eri.assign(d.eri, d.eri + (size_t)n * n * n * n);
        // exact copies of the integrals the diagonal element reads
        s.hd.resize(n);
        s.Jt.resize((size_t)n * n);
        s.Kt.resize((size_t)n * n);
        for (int p = 0; p < n; ++p) {
            s.hd[p] = s.h1[(size_t)p * n + p];
            for (int q = 0; q < n; ++q) {
                s.Jt[(size_t)p * n + q] = s.eri[(((size_t)p * n + p) * n + q) * n + q];
                s.Kt[(size_t)p * n + q] = s.eri[(((size_t)p * n + q) * n + q) * n + p];
            }
        }
        for (int i = 0; i < d.n_alpha; ++i) setbit_h(s.ref, 2 * i);
        for (int i = 0; i < d.n_beta; ++i) setbit_h(s.ref, 2 * i + 1);
        const int ns = 2 * n;
        s.hb_off.assign((size_t)ns * ns, 0);
        s.hb_cnt.assign((size_t)ns * ns, 0);
        s.hb_S.assign((size_t)ns * ns, 0.0);
        // heat-bath tables: allowed A < B (spin conserving, outside {P,Q}) in
        // lexicographic order, weight |<AB|PQ> - <AB|QP>|, sequential running sums
        int64_t tot = 0;
        for (int P = 0; P < ns; ++P)
            for (int Q = P + 1; Q < ns; ++Q) {
                s.hb_off[(size_t)P * ns + Q] = tot;
                double cum = 0.0;
                int cnt = 0;
                for (int A = 0; A < ns; ++A)
                    for (int B = A + 1; B < ns; ++B) {
                        if (A == P || A == Q || B == P || B == Q) continue;
                        if ((A & 1) + (B & 1) != (P & 1) + (Q & 1)) continue;
                        cum = cum + std::fabs(antisym_mol(s, A, B, P, Q));
                        s.hb_AB.push_back((uint16_t)(A | (B << 8)));
                        s.hb_cdf.push_back(cum);
                        ++cnt;
                    }
                s.hb_cnt[(size_t)P * ns + Q] = cnt;
                s.hb_S[(size_t)P * ns + Q] = cum;
                tot += cnt;
            }
    } else {
        return "unknown system kind";
    }
    s.n_so = 2 * s.n_spatial;
    return "";
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// device image of one system's tables
size_t table_bytes(const HostSys &s)
{
    return al(4 * s.npk.size()) + al(8 * s.eps.size()) + al(8 * s.vtab.size()) + al(8 * s.vx.size()) + al(2 * s.grid.size()) +
           al(8 * s.h1.size()) + al(8 * s.eri.size()) + al(8 * s.hd.size()) + al(8 * s.Jt.size()) + al(8 * s.Kt.size()) + al(8 * s.hb_off.size()) + al(4 * s.hb_cnt.size()) +
           al(8 * s.hb_S.size()) + al(2 * s.hb_AB.size()) + al(8 * s.hb_cdf.size());
}

struct Layout {
    size_t total = 0;
    size_t ctl, acc, hist, shift, rep, sys, tables, att, span, mpart, st_scan, st_sort, st_red, st_merge, st_att;
    size_t part_red, part_mrg, newdet, bpart;
    size_t main[2][6];
    size_t sp[7];
    size_t u[4];
    size_t ds[14];
    size_t dkeys;
    size_t cc_cum, st_ccmc, single_key, single_pop;  // CCMC (empty otherwise)
};

int64_t tiles_of(int64_t n, int64_t tile) { return (n + tile - 1) / tile + 1; }

// the density-matrix methods key pairs of determinants
bool dm_method(int m) { return m == FQ_DMQMC || m == FQ_IPDMQMC; }

// CCMC: room for every single excitation of the reference (the queue of
// singles of the projected energy); 0 for the other methods
int64_t single_capacity(const HostSys &s, int method)
{
    if (method != FQ_CCMC) return 0;
    return (int64_t)s.na * (s.n_spatial - s.na) + (int64_t)s.nb * (s.n_spatial - s.nb) + 1;
}

// two descriptions of the same Hamiltonian (integral arrays compared by value)
bool same_system(const fq_system &a, const fq_system &b)
{
    if (a.kind != b.kind || a.n_alpha != b.n_alpha || a.n_beta != b.n_beta) return false;
    if (a.kind == FQ_HUBBARD_REAL)
        return a.n_sites == b.n_sites && a.periodic == b.periodic && a.t == b.t && a.U == b.U;
    if (a.kind == FQ_UEG) return a.rs == b.rs && a.ecut_n2 == b.ecut_n2;
    if (a.n_orb != b.n_orb || !a.h1 || !b.h1 || !a.eri || !b.eri) return false;
    const size_t n2 = (size_t)a.n_orb * a.n_orb;
    return std::memcmp(a.h1, b.h1, 8 * n2) == 0 && std::memcmp(a.eri, b.eri, 8 * n2 * n2) == 0;
}

// spans of 256 attempts the attempt partition can hold
int64_t span_capacity(int64_t mcap, int64_t scap, int W)
{
    (void)W;
    return tiles_of(std::max(mcap * 16, scap * 4), SPAN_MIN);
}

Layout make_layout(int R, int W, int64_t mcap, int64_t scap, int64_t tables, int D, int nk, int64_t singles)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += al(b);
        return r;
    };
    L.ctl = take(sizeof(Ctl));
    L.acc = take(sizeof(EstAcc) * R);
    L.hist = take(sizeof(EstAcc) * R * HIST_LEN);
    L.shift = take(8 * R);
    L.rep = take(sizeof(RepParams) * R);
    L.sys = take(sizeof(DevSys) * R);
    L.tables = take((size_t)tables);
    L.att = take(8 * (size_t)(mcap + 1));
    L.span = take(8 * (size_t)(span_capacity(mcap, scap, W) + 2));
    L.mpart = take(8 * (size_t)(tiles_of(mcap + scap, 512) + 2));
    L.newdet = take((size_t)mcap + 16);
    L.bpart = take(sizeof(BoundaryPart) * (size_t)tiles_of(scap, 1024));
    L.st_scan = take(8 * (size_t)tiles_of(mcap, 2048));
    L.st_sort = take(8 * 256 * (size_t)tiles_of(scap, SORT_TILE_MIN));
    L.st_red = take(8 * (size_t)tiles_of(scap, 1024));
    L.st_merge = take(8 * (size_t)tiles_of(mcap + scap, 512));
    L.st_att = take(8 * (size_t)tiles_of(mcap + scap, 512));
    L.part_red = take(8 * (size_t)PART_MAX_BLOCKS * acc_rows(R) * EST_FIELDS);
    L.part_mrg = take(8 * (size_t)PART_MAX_BLOCKS * acc_rows(R) * EST_FIELDS);
    for (int b = 0; b < 2; ++b) {
        L.main[b][0] = take(8 * (size_t)mcap);
        L.main[b][1] = take(8 * (size_t)mcap * W);
        L.main[b][2] = take(4 * (size_t)mcap);
        L.main[b][3] = take(8 * (size_t)mcap);
        L.main[b][4] = take(4 * (size_t)mcap);
        L.main[b][5] = take(4 * (size_t)mcap);
    }
    L.sp[0] = take(8 * (size_t)scap);
    L.sp[1] = take(8 * (size_t)scap * (W + 1));
    L.sp[2] = take(0);
    L.sp[3] = take(0);
    L.sp[4] = take(8 * (size_t)scap);
    L.sp[5] = take(4 * (size_t)scap);
    L.sp[6] = take(4 * (size_t)scap);
    L.u[0] = take(8 * (size_t)scap);
    L.u[1] = take(8 * (size_t)scap * W);
    L.u[2] = take(8 * (size_t)scap);
    L.u[3] = take(4 * (size_t)scap);
    const size_t nd = (size_t)D * R;
    const size_t np = (size_t)((D + 31) / 32) * 32;  // MFMA k steps of 32
    L.ds[0] = take(8 * (size_t)nk * D * (size_t)D);  // K fp64
    L.ds[1] = take(2 * (size_t)nk * np * np);        // K hi bf16
    L.ds[2] = take(2 * (size_t)nk * np * np);        // K lo bf16
    L.ds[3] = take(4 * nd);              // pos
    L.ds[4] = take(8 * nd);              // h64
    L.ds[5] = take(8 * nd);              // c
    L.ds[6] = take(8 * nd);              // y
    L.ds[7] = take(8 * nd);              // delta
    L.ds[8] = take(8 * nd);              // sorted skeys
    L.ds[9] = take(8 * nd * W);          // sorted keys
    L.ds[10] = take(2 * (size_t)R * np); // c hi bf16
    L.ds[11] = take(2 * (size_t)R * np); // c lo bf16
    L.ds[12] = take(8 * nd);             // FP64 reference y
    L.dkeys = take(8 * nd * W);          // keys in D order
    const bool cc = singles > 0;
    L.cc_cum = take(cc ? 8 * (size_t)(mcap + 1) : 0);
    L.st_ccmc = take(cc ? 8 * (size_t)tiles_of(mcap, 2048) : 0);
    L.single_key = take(8 * (size_t)singles * W);
    L.single_pop = take(4 * (size_t)singles);
    L.total = o;
    return L;
}

}  // namespace

struct fq_ctx {
    int R = 0, W = 0, kind = 0, rb = 0;
    int method = FQ_FCIQMC;  // FQ_FCIQMC, FQ_DMQMC, FQ_IPDMQMC or FQ_CCMC (one per context)
    int lkind = 0;           // kernel kind: the system kind, | K_PAIR for the density-matrix methods
    uint64_t hmask = ~0ull;  // hash bits that enter a sort key
    hipStream_t stream = nullptr;
    std::vector<HostSys> sys;
    std::vector<fq_qmc> qmc;
    bool has_ss = false;
    fq_semistoch ss{};
    int D = 0;
    bool ss_active = false;
    Layout L;
    char *ws = nullptr;
    Work w{};
    MainList buf[2];
    int cur = 0;
    int64_t main_cap = 0, spawn_cap = 0;
    Grids grids{};
    std::vector<double> shift;
    std::vector<int> vary;
    std::vector<int64_t> nprev;
    int64_t t = 0;           // completed (enqueued and synchronised) iterations
    std::vector<fq_estimators_t> last;
    std::vector<std::vector<fq_estimators_t>> hist;  // [R][...] of the last fq_step
    std::vector<std::vector<uint64_t>> dkeys;        // [R][D*W] D order
    Ctl *h_ctl = nullptr;
    EstAcc *h_hist = nullptr;
    double *h_shift = nullptr;
    double h00[64] = {0};
    std::vector<double> rs_max;  // [R] time-step search: largest |H_ji| / p_gen so far
    std::vector<double> h00v;
    bool timing = false;
    bool graph = false;
    hipGraph_t graphs[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_len[2] = {0, 0};
    double stage_ms[7] = {0};
    double kernel_ms[N_KERNEL_SLOTS] = {0};
    int64_t timed_iterations = 0;
    std::vector<double> iter_ms;  // per-iteration device time of the last timed fq_step
    std::string err;
    bool pinned = true;   // host staging buffers from hipHostMalloc (else plain host memory)
    int static_dev = -1;  // device whose static workspace array this context holds (-1: none)
};

namespace {

// Every copy and fill of a context is ordered on the context's stream (the
// caller's stream need not synchronise with the legacy default stream); the
// host waits for the stream before it reads a result or lets a host buffer go.
hipError_t h2d(hipStream_t s, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

hipError_t d2h(hipStream_t s, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

hipError_t fill0(hipStream_t s, void *dst, size_t bytes)
{
    return hipMemsetAsync(dst, 0, bytes, s);
}

fq_status fail(fq_ctx *c, fq_status s, const std::string &m)
{
    if (c) c->err = m;
    return s;
}

#define HIPCHK(ctx, call)                                                                \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(ctx, FQ_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

void estimators_from_acc(const fq_ctx *c, int r, const EstAcc &a, fq_estimators_t &e)
{
    std::memset(&e, 0, sizeof(e));
    e.iteration = a.t;
    e.n_walkers_units = a.nw;
    e.n_occupied = a.nocc;
    e.n_spawned = a.nspawn;
    e.ref_pop_units = a.n0;
    e.n_sign_flips = a.flips;
    e.n_rejected_units = a.rej_units;
    e.n_spawn_events = a.nuniq;
    e.death_sum = a.death_sum;
    e.spawn_sum = a.spawn_sum;
    e.rejected_sum = a.rej_sum;
    for (int k = 0; k < 4; ++k) e.num_limbs[k] = a.limbs[k];
    for (int k = 0; k < 4; ++k) e.pair_limbs[k] = a.pair[k];
    e.n_cluster_spawns = a.ccmc_rec;
    e.ss_error = a.ss_err;
    if (c->has_ss && c->ss.precision == FQ_SS_SPLIT_BF16)
        e.ss_error_bound = 3.0 * 0x1p-16 + 3.0 * (double)c->D * 0x1p-24;
    __int128 tot = 0;
    for (int k = 0; k < 4; ++k) tot += (__int128)a.limbs[k] * ((__int128)1 << (32 * k));
    double num = (double)tot * 0x1p-64;
    if (c->method == FQ_CCMC && a.n0 != 0) {
        // t~_j of the doubles holds the products of pairs of singles over N_0
        __int128 pt = 0;
        for (int k = 0; k < 4; ++k) pt += (__int128)a.pair[k] * ((__int128)1 << (32 * k));
        num = num + ((double)pt * 0x1p-64) / (double)a.n0;
    }
    e.proj_numerator = num * std::ldexp(1.0, -c->qmc[r].fixed_point_bits);
    e.proj_energy = a.n0 != 0 ? num / (double)a.n0 : NAN;
    e.e_ref = c->h00v[r];
    e.tau = c->qmc[r].tau;
    e.spawn_ratio_max = c->rs_max[r];
}

// time-step search: fold the per-iteration maxima of |H_ji| / p_gen of
// iterations first..last (held in the host copy of the history ring) into each
// replica's running maximum
void fold_spawn_ratio(fq_ctx *c, int64_t first, int64_t last)
{
    for (int64_t it = first; it <= last; ++it)
        for (int r = 0; r < c->R; ++r) {
            const unsigned long long b = c->h_hist[(size_t)(it % HIST_LEN) * c->R + r].rs_bits;
            double v;
            std::memcpy(&v, &b, 8);
            if (v > c->rs_max[r]) c->rs_max[r] = v;
        }
}

void set_main_views(fq_ctx *c)
{
    for (int b = 0; b < 2; ++b) {
        MainList &m = c->buf[b];
        m.skey = (uint64_t *)(c->ws + c->L.main[b][0]);
        m.key = (uint64_t *)(c->ws + c->L.main[b][1]);
        m.pop = (int32_t *)(c->ws + c->L.main[b][2]);
        m.kdiag = (double *)(c->ws + c->L.main[b][3]);
        m.dslot = (int32_t *)(c->ws + c->L.main[b][4]);
        m.natt = (int32_t *)(c->ws + c->L.main[b][5]);
    }
    c->w.cur = c->buf[c->cur];
    c->w.nxt = c->buf[c->cur ^ 1];
}

void drop_graphs(fq_ctx *c)
{
    for (int b = 0; b < 2; ++b) {
        if (c->gexec[b]) (void)hipGraphExecDestroy(c->gexec[b]);
        if (c->graphs[b]) (void)hipGraphDestroy(c->graphs[b]);
        c->gexec[b] = nullptr;
        c->graphs[b] = nullptr;
        c->graph_len[b] = 0;
    }
}

struct HostEntry {
    uint64_t skey;
    uint64_t key[MAXW];
    int32_t pop;
    int32_t dslot;
};

// downloads the whole current main list
fq_status download_main(fq_ctx *c, std::vector<HostEntry> &out, int64_t &n)
{
    HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    n = c->h_ctl->n_main_new;
    const MainList &m = c->buf[c->cur];
    std::vector<uint64_t> sk(n), kk((size_t)n * c->W);
    std::vector<int32_t> pp(n), ds(n);
    // sort keys not kept by the kernels are the keys' hashes
    const bool stored = stored_skey(c->R > 1, c->W);
    if (n) {
        if (stored) HIPCHK(c, d2h(c->stream, sk.data(), m.skey, 8 * n));
        for (int q = 0; q < c->W; ++q)
            HIPCHK(c, d2h(c->stream, kk.data() + (size_t)q * n, m.key + (size_t)q * c->main_cap, 8 * n));
        HIPCHK(c, d2h(c->stream, pp.data(), m.pop, 4 * n));
        HIPCHK(c, d2h(c->stream, ds.data(), m.dslot, 4 * n));
    }
    out.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < MAXW; ++q) out[i].key[q] = q < c->W ? kk[(size_t)q * n + i] : 0;
        out[i].skey = stored ? sk[i] : host_skey(host_hash(out[i].key, c->W) & c->hmask, 0u, c->rb);
        out[i].pop = pp[i];
        out[i].dslot = ds[i];
    }
    return FQ_OK;
}

// uploads a list sorted by (skey, key) into the current buffer, recomputes
// K_ii - H_00 and attempt counts on the device
fq_status upload_main(fq_ctx *c, const std::vector<HostEntry> &e)
{
    const int64_t n = (int64_t)e.size();
    if (n > c->main_cap) return fail(c, FQ_ECAPACITY, "main list capacity exceeded");
    drop_graphs(c);  // captured blocks are rebuilt from the current state on the next step
    const MainList &m = c->buf[c->cur];
    std::vector<uint64_t> sk(n), kk((size_t)n * c->W);
    std::vector<int32_t> pp(n), ds(n);
    for (int64_t i = 0; i < n; ++i) {
        sk[i] = e[i].skey;
        for (int q = 0; q < c->W; ++q) kk[(size_t)q * n + i] = e[i].key[q];
        pp[i] = e[i].pop;
        ds[i] = e[i].dslot;
    }
    if (n) {
        HIPCHK(c, h2d(c->stream, m.skey, sk.data(), 8 * n));
        for (int q = 0; q < c->W; ++q)
            HIPCHK(c, h2d(c->stream, m.key + (size_t)q * c->main_cap, kk.data() + (size_t)q * n, 8 * n));
        HIPCHK(c, h2d(c->stream, m.pop, pp.data(), 4 * n));
        HIPCHK(c, h2d(c->stream, m.dslot, ds.data(), 4 * n));
    }
    set_main_views(c);
    {
        Ctl ctl0;
        HIPCHK(c, d2h(c->stream, &ctl0, c->w.ctl, sizeof(Ctl)));
        ctl0.n_main = n;
        ctl0.n_main_new = n;
        std::memset(ctl0.tickets, 0, sizeof(ctl0.tickets));
        HIPCHK(c, h2d(c->stream, c->w.ctl, &ctl0, sizeof(Ctl)));
    }
    // every look-back status array: an import may set the iteration counter
    // back, and a rollback re-runs the failed iteration, so words of an
    // earlier pass could carry the epoch the next iterations use
    HIPCHK(c, fill0(c->stream, c->ws + c->L.st_scan, c->L.part_red - c->L.st_scan));
    if (c->L.single_key > c->L.st_ccmc)
        HIPCHK(c, fill0(c->stream, c->ws + c->L.st_ccmc, c->L.single_key - c->L.st_ccmc));
    HIPCHK(c, enqueue_setup(1, c->lkind, c->w, nullptr, 0, m, n, nullptr, nullptr, c->stream));
    Ctl ctl;
    HIPCHK(c, d2h(c->stream, &ctl, c->w.ctl, sizeof(Ctl)));
    ctl.n_main = n;
    ctl.n_main_new = n;
    HIPCHK(c, h2d(c->stream, c->w.ctl, &ctl, sizeof(Ctl)));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FQ_OK;
}

bool entry_less(const HostEntry &a, const HostEntry &b, int W)
{
    if (a.skey != b.skey) return a.skey < b.skey;
    return key_cmp_host(a.key, b.key, W) < 0;
}

// initial estimators of each replica (iteration counter value, list as is)
fq_status host_estimators(fq_ctx *c)
{
    std::vector<HostEntry> e;
    int64_t n;
    fq_status st = download_main(c, e, n);
    if (st) return st;
    for (int r = 0; r < c->R; ++r) {
        EstAcc a;
        std::memset(&a, 0, sizeof(a));
        a.t = c->t;
        for (const HostEntry &x : e) {
            const uint32_t rep = c->rb ? (uint32_t)(x.skey >> (64 - c->rb)) : 0u;
            if ((int)rep != r) continue;
            a.nw += x.pop < 0 ? -(long long)x.pop : x.pop;
            a.nocc += 1;
            if (dm_method(c->method)) {
                if (x.key[0] == x.key[1]) a.n0 += x.pop;  // the trace
            } else if (key_cmp_host(x.key, c->sys[r].ref, c->W) == 0) {
                a.n0 = x.pop;
            }
        }
        if (c->method == FQ_CCMC) {
            // the singles-pair part of the projected energy, on the device
            HIPCHK(c, fill0(c->stream, &c->w.acc[0], sizeof(EstAcc)));
            HIPCHK(c, fill0(c->stream, (char *)c->w.ctl + offsetof(Ctl, n_single), sizeof(uint32_t)));
            HIPCHK(c, enqueue_ccmc(2, c->lkind, c->w, c->grids, c->stream));
            EstAcc dv;
            HIPCHK(c, d2h(c->stream, &dv, &c->w.acc[0], sizeof(EstAcc)));
            for (int k = 0; k < 4; ++k) a.pair[k] = dv.pair[k];
        }
        estimators_from_acc(c, r, a, c->last[r]);
        c->last[r].shift = c->shift[r];
        c->last[r].vary_shift = c->vary[r];
    }
    return FQ_OK;
}

// deterministic space: the `size` largest |n| of each replica (key ascending on ties)
fq_status select_detspace(fq_ctx *c)
{
    std::vector<HostEntry> e;
    int64_t n;
    fq_status st = download_main(c, e, n);
    if (st) return st;
    const int D = c->D, R = c->R, W = c->W;
    const size_t nd = (size_t)D * R;
    std::vector<int32_t> pos(nd, 0);
    std::vector<uint64_t> h64(nd, 0), dk(nd * W, 0);
    c->dkeys.assign(R, std::vector<uint64_t>((size_t)D * W, 0));
    auto rep_of = [&](const HostEntry &x) { return c->rb ? (uint32_t)(x.skey >> (64 - c->rb)) : 0u; };
    if (!c->ss.shared) {
        // each replica: its D most highly weighted determinants
        for (int r = 0; r < R; ++r) {
            std::vector<int64_t> ix;
            for (int64_t i = 0; i < n; ++i)
                if ((int)rep_of(e[i]) == r) ix.push_back(i);
            if ((int64_t)ix.size() < D)
                return fail(c, FQ_ESTATE, "fewer occupied determinants than the deterministic space size");
            std::partial_sort(ix.begin(), ix.begin() + D, ix.end(), [&](int64_t a, int64_t b) {
                const long long pa = std::llabs((long long)e[a].pop), pb = std::llabs((long long)e[b].pop);
                if (pa != pb) return pa > pb;
                return key_cmp_host(e[a].key, e[b].key, W) < 0;
            });
            for (int d = 0; d < D; ++d)
                for (int q = 0; q < W; ++q) c->dkeys[r][(size_t)d * W + q] = e[ix[d]].key[q];
        }
    } else {
        // one D for all replicas: largest summed |n| over the replicas, key
        // ascending on ties
        std::vector<int64_t> ix(n);
        std::iota(ix.begin(), ix.end(), 0);
        std::sort(ix.begin(), ix.end(), [&](int64_t a, int64_t b) { return key_cmp_host(e[a].key, e[b].key, W) < 0; });
        std::vector<std::pair<int64_t, int64_t>> tot;  // (summed |n|, entry holding the key)
        for (int64_t x = 0; x < n; ++x) {
            const int64_t i = ix[x];
            const int64_t a = std::llabs((long long)e[i].pop);
            if (!tot.empty() && key_cmp_host(e[tot.back().second].key, e[i].key, W) == 0)
                tot.back().first += a;
            else
                tot.push_back({a, i});
        }
        if ((int64_t)tot.size() < D)
            return fail(c, FQ_ESTATE, "fewer occupied determinants than the deterministic space size");
        std::sort(tot.begin(), tot.end(), [&](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
            if (a.first != b.first) return a.first > b.first;
            return key_cmp_host(e[a.second].key, e[b.second].key, W) < 0;
        });
        for (int r = 0; r < R; ++r)
            for (int d = 0; d < D; ++d)
                for (int q = 0; q < W; ++q) c->dkeys[r][(size_t)d * W + q] = e[tot[d].second].key[q];
        // every replica holds every member: the missing ones enter with n = 0
        std::vector<HostEntry> add;
        for (int r = 0; r < R; ++r)
            for (int d = 0; d < D; ++d) {
                HostEntry x;
                std::memset(&x, 0, sizeof(x));
                for (int q = 0; q < W; ++q) x.key[q] = c->dkeys[r][(size_t)d * W + q];
                x.skey = host_skey(host_hash(x.key, W) & c->hmask, (uint32_t)r, c->rb);
                x.dslot = -1;
                auto it = std::lower_bound(e.begin(), e.end(), x,
                                           [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, W); });
                if (it == e.end() || it->skey != x.skey || key_cmp_host(it->key, x.key, W) != 0) add.push_back(x);
            }
        if (!add.empty()) {
            if (n + (int64_t)add.size() > c->main_cap) return fail(c, FQ_ECAPACITY, "main list capacity exceeded");
            e.insert(e.end(), add.begin(), add.end());
            std::sort(e.begin(), e.end(), [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, W); });
            n = (int64_t)e.size();
        }
    }
    // slots and positions of the members in the (sorted) list
    for (auto &x : e) x.dslot = -1;
    for (int r = 0; r < R; ++r)
        for (int d = 0; d < D; ++d) {
            HostEntry x;
            std::memset(&x, 0, sizeof(x));
            for (int q = 0; q < W; ++q) x.key[q] = c->dkeys[r][(size_t)d * W + q];
            x.skey = host_skey(host_hash(x.key, W) & c->hmask, (uint32_t)r, c->rb);
            auto it = std::lower_bound(e.begin(), e.end(), x,
                                       [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, W); });
            const int64_t i = it - e.begin();
            e[i].dslot = d;
            pos[(size_t)r * D + d] = (int32_t)i;
            h64[(size_t)r * D + d] = host_hash(x.key, W);
            for (int q = 0; q < W; ++q) dk[(size_t)q * nd + (size_t)r * D + d] = x.key[q];
        }
    // sorted copy for membership tests
    std::vector<size_t> order(nd);
    std::iota(order.begin(), order.end(), 0);
    std::vector<uint64_t> sks(nd);
    for (size_t x = 0; x < nd; ++x) {
        uint64_t k[MAXW] = {0};
        for (int q = 0; q < W; ++q) k[q] = dk[(size_t)q * nd + x];
        sks[x] = host_skey(host_hash(k, W) & c->hmask, (uint32_t)(x / D), c->rb);
    }
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (sks[a] != sks[b]) return sks[a] < sks[b];
        uint64_t ka[MAXW] = {0}, kb[MAXW] = {0};
        for (int q = 0; q < W; ++q) {
            ka[q] = dk[(size_t)q * nd + a];
            kb[q] = dk[(size_t)q * nd + b];
        }
        return key_cmp_host(ka, kb, W) < 0;
    });
    std::vector<uint64_t> ssk(nd), skk(nd * W);
    for (size_t x = 0; x < nd; ++x) {
        ssk[x] = sks[order[x]];
        for (int q = 0; q < W; ++q) skk[(size_t)q * nd + x] = dk[(size_t)q * nd + order[x]];
    }
    // dslot of the current list (with the members added to it, the whole list)
    const MainList &m = c->buf[c->cur];
    if (c->ss.shared) {
        fq_status su = upload_main(c, e);
        if (su) return su;
    } else {
        std::vector<int32_t> ds(n);
        for (int64_t i = 0; i < n; ++i) ds[i] = e[i].dslot;
        if (n) HIPCHK(c, h2d(c->stream, m.dslot, ds.data(), 4 * n));
    }
    HIPCHK(c, h2d(c->stream, c->ws + c->L.ds[3], pos.data(), 4 * nd));
    HIPCHK(c, h2d(c->stream, c->ws + c->L.ds[4], h64.data(), 8 * nd));
    HIPCHK(c, h2d(c->stream, c->ws + c->L.ds[8], ssk.data(), 8 * nd));
    HIPCHK(c, h2d(c->stream, c->ws + c->L.ds[9], skk.data(), 8 * nd * W));
    HIPCHK(c, h2d(c->stream, c->ws + c->L.dkeys, dk.data(), 8 * nd * W));
    HIPCHK(c, fill0(c->stream, c->ws + c->L.ds[6], 8 * nd));
    HIPCHK(c, enqueue_setup(2, c->lkind, c->w, nullptr, 0, m, 0, (const uint64_t *)(c->ws + c->L.dkeys),
                            (double *)(c->ws + c->L.ds[0]), c->stream));
    Ctl ctl;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, d2h(c->stream, &ctl, c->w.ctl, sizeof(Ctl)));
    ctl.ss_active = 1;
    HIPCHK(c, h2d(c->stream, c->w.ctl, &ctl, sizeof(Ctl)));
    c->ss_active = true;
    return FQ_OK;
}

}  // namespace

extern "C" {

size_t fq_workspace_bytes(const fq_system *sys, const fq_qmc *qmc, const fq_semistoch *ss, int32_t n_instances,
                          int64_t main_capacity, int64_t spawn_capacity)
{
    if (!sys || n_instances <= 0 || main_capacity <= 0 || spawn_capacity <= 0) return 0;
    int64_t tables = 0, singles = 0;
    int W = 1;
    for (int r = 0; r < n_instances; ++r) {
        HostSys s;
        if (!build_system(sys[r], s).empty()) return 0;
        tables += (int64_t)table_bytes(s);
        const int pair = qmc && dm_method(qmc[r].method) ? 2 : 1;
        W = std::max(W, pair * round_w(s.n_so));
        singles = std::max(singles, single_capacity(s, qmc ? qmc[r].method : FQ_FCIQMC));
    }
    const int D = ss ? std::max(0, ss[0].size) : 0;
    const int nk = ss && ss[0].shared ? 1 : n_instances;
    return make_layout(n_instances, W, main_capacity, spawn_capacity, tables, D, nk, singles).total + 256;
}

}  // extern "C"

namespace {

// Body of the two set-up entry points. pinned: stage estimators and counters
// through page-locked host buffers (hipHostMalloc); otherwise through plain
// host memory, so that the call allocates nothing through HIP.
fq_status init_system(fq_ctx **out, const fq_system *sys, const fq_qmc *qmc, const fq_semistoch *ss,
                      int32_t n_instances, int64_t main_capacity, int64_t spawn_capacity, void *d_workspace,
                      size_t ws_bytes, void *hip_stream, bool pinned, int static_dev)
{
    if (!out || !sys || !qmc || n_instances <= 0 || n_instances > 4096 || main_capacity < n_instances ||
        spawn_capacity < 1 || !d_workspace)
        return FQ_EINVAL;
    if (spawn_capacity >= (1ll << 32)) return FQ_EINVAL;
    for (int r = 0; r < n_instances; ++r)
    *out = nullptr;
    fq_ctx *c = new fq_ctx();
    c->pinned = pinned;
    c->R = n_instances;
    c->stream = (hipStream_t)hip_stream;
    c->main_cap = main_capacity;
    c->spawn_cap = spawn_capacity;
    c->sys.resize(c->R);
    c->qmc.assign(qmc, qmc + c->R);
    int64_t tables = 0;
    for (int r = 0; r < c->R; ++r) {
        const std::string m = build_system(sys[r], c->sys[r]);
        if (!m.empty()) { delete c; return FQ_EINVAL; }
        // density-matrix methods: a key holds a pair of one-word determinants
        const int Wd = round_w(c->sys[r].n_so);
        const int W = dm_method(qmc[r].method) ? 2 * Wd : Wd;
        if (r == 0) { c->W = W; c->kind = sys[r].kind; c->method = qmc[0].method; }
        if (W != c->W || sys[r].kind != c->kind || qmc[r].method != c->method) { delete c; return FQ_EINVAL; }
        if (qmc[r].method < FQ_FCIQMC || qmc[r].method > FQ_CCMC) { delete c; return FQ_EINVAL; }
        if (dm_method(qmc[r].method) &&
            (Wd != 1 || qmc[r].initiator || qmc[r].tau_search || (ss && ss[0].size > 0)))
            { delete c; return FQ_EINVAL; }
        // CCMC: one instance, excitors of level 1..6, no initiator rule,
        // deterministic space or time-step search
        if (qmc[r].method == FQ_CCMC &&
            (n_instances != 1 || qmc[r].ccmc_truncation < 1 || qmc[r].ccmc_truncation > 6 || qmc[r].initiator ||
             qmc[r].tau_search || (ss && ss[0].size > 0)))
            { delete c; return FQ_EINVAL; }
        const fq_qmc &q = qmc[r];
        const int need = c->kind == FQ_HUBBARD_REAL ? FQ_EXGEN_HUB_UNIFORM
                         : c->kind == FQ_UEG        ? FQ_EXGEN_UEG_UNIFORM
                                                    : FQ_EXGEN_HEATBATH_UNIFORM_SINGLES;
        // fixed_point_bits 1 and 2 would allow 2^28 or more attempts on one
        // determinant (int32 populations), beyond the attempt field of the
        // random-number counter
        if (!(q.tau > 0) || q.excit_gen != need || q.fixed_point_bits < 0 || q.fixed_point_bits > 20 ||
            (q.fixed_point_bits > 0 && q.fixed_point_bits < 3) ||
            q.shift_period <= 0 || q.shift_period > HIST_LEN / 2 || !(q.init_pop >= 0) ||
            (q.excit_gen == FQ_EXGEN_HEATBATH_UNIFORM_SINGLES && !(q.p_single >= 0 && q.p_single < 1))) {
            delete c;
            return FQ_EINVAL;
        }
        tables += (int64_t)table_bytes(c->sys[r]);
    }
    if (c->kind == FQ_HUBBARD_REAL && c->W != (dm_method(c->method) ? 2 : 1)) { delete c; return FQ_EINVAL; }
    c->lkind = c->kind | (dm_method(c->method) ? (int)K_PAIR : 0);
    for (int r = 1; r < c->R; ++r)
        if (qmc[r].shift_period != qmc[0].shift_period) { delete c; return FQ_EINVAL; }
    c->rb = 0;
    while ((1 << c->rb) < c->R) ++c->rb;
    if (ss && ss[0].size > 0) {
        c->has_ss = true;
        c->ss = ss[0];
        c->D = ss[0].size;
        if (ss[0].precision != FQ_SS_FP64 && ss[0].precision != FQ_SS_SPLIT_BF16) { delete c; return FQ_EINVAL; }
        for (int r = 1; r < c->R; ++r)
            if (ss[r].size != ss[0].size || ss[r].start_iteration != ss[0].start_iteration ||
                ss[r].shared != ss[0].shared)
                { delete c; return FQ_EINVAL; }
        if (ss[0].shared != 0 && ss[0].shared != 1) { delete c; return FQ_EINVAL; }
        // one deterministic space for all instances needs one Hamiltonian
        if (ss[0].shared)
            for (int r = 1; r < c->R; ++r)
                if (!same_system(sys[0], sys[r])) { delete c; return FQ_EINVAL; }
    }
    const int nk = c->has_ss && c->ss.shared ? 1 : c->R;
    const int64_t singles = single_capacity(c->sys[0], c->method);
    c->L = make_layout(c->R, c->W, main_capacity, spawn_capacity, tables, c->D, nk, singles);
    if (ws_bytes < c->L.total || ((uintptr_t)d_workspace & 255)) { delete c; return FQ_EINVAL; }
    c->ws = (char *)d_workspace;
    Work &w = c->w;
    w.ctl = (Ctl *)(c->ws + c->L.ctl);
    w.acc = (EstAcc *)(c->ws + c->L.acc);
    w.hist = (EstAcc *)(c->ws + c->L.hist);
    w.shift = (double *)(c->ws + c->L.shift);
    w.rep = (const RepParams *)(c->ws + c->L.rep);
    w.sys = (const DevSys *)(c->ws + c->L.sys);
    w.att_off = (long long *)(c->ws + c->L.att);
    w.span_lo = (long long *)(c->ws + c->L.span);
    w.mpart = (long long *)(c->ws + c->L.mpart);
    w.newdet = (uint8_t *)(c->ws + c->L.newdet);
    w.bpart = (BoundaryPart *)(c->ws + c->L.bpart);
    w.st_scan = (unsigned long long *)(c->ws + c->L.st_scan);
    w.st_sort = (unsigned long long *)(c->ws + c->L.st_sort);
    w.st_red = (unsigned long long *)(c->ws + c->L.st_red);
    w.st_merge = (unsigned long long *)(c->ws + c->L.st_merge);
    w.st_att = (unsigned long long *)(c->ws + c->L.st_att);
    w.part_red = (long long *)(c->ws + c->L.part_red);
    w.part_mrg = (long long *)(c->ws + c->L.part_mrg);
    w.sp.skey = (uint64_t *)(c->ws + c->L.sp[0]);
    w.sp.rec = (uint64_t *)(c->ws + c->L.sp[1]);
    w.sp.skey2 = (uint64_t *)(c->ws + c->L.sp[4]);
    w.sp.idx = (uint32_t *)(c->ws + c->L.sp[5]);
    w.sp.idx2 = (uint32_t *)(c->ws + c->L.sp[6]);
    w.u.skey = (uint64_t *)(c->ws + c->L.u[0]);
    w.u.key = (uint64_t *)(c->ws + c->L.u[1]);
    w.u.sum = (long long *)(c->ws + c->L.u[2]);
    w.u.flag = (uint32_t *)(c->ws + c->L.u[3]);
    w.ds.n = c->D;
    w.ds.precision = c->has_ss ? c->ss.precision : 0;
    w.ds.K = (const double *)(c->ws + c->L.ds[0]);
    w.ds.npad = ((c->D + 31) / 32) * 32;
    w.ds.check_period = c->has_ss ? c->ss.check_period : 0;
    w.ds.shared = c->has_ss ? c->ss.shared : 0;
    w.ds.nk = nk;
    w.ds.Khi = (uint16_t *)(c->ws + c->L.ds[1]);
    w.ds.Klo = (uint16_t *)(c->ws + c->L.ds[2]);
    w.ds.Chi = (uint16_t *)(c->ws + c->L.ds[10]);
    w.ds.Clo = (uint16_t *)(c->ws + c->L.ds[11]);
    w.ds.yref = (double *)(c->ws + c->L.ds[12]);
    w.ds.pos = (int32_t *)(c->ws + c->L.ds[3]);
    w.ds.h64 = (const uint64_t *)(c->ws + c->L.ds[4]);
    w.ds.c = (double *)(c->ws + c->L.ds[5]);
    w.ds.y = (double *)(c->ws + c->L.ds[6]);
    w.ds.delta = (long long *)(c->ws + c->L.ds[7]);
    w.ds.skey_sorted = (const uint64_t *)(c->ws + c->L.ds[8]);
    w.ds.key_sorted = (const uint64_t *)(c->ws + c->L.ds[9]);
    w.main_cap = main_capacity;
    w.spawn_cap = spawn_capacity;
    w.span_cap = span_capacity(main_capacity, spawn_capacity, c->W);
    w.R = c->R;
    w.rb = c->rb;
    w.hmask = c->hmask;
    w.tau_search = c->qmc[0].tau_search;
    w.dm = dm_method(c->method) ? c->method : 0;
    w.ccmc_trunc = c->method == FQ_CCMC ? c->qmc[0].ccmc_truncation : 0;
    w.single_cap = (int32_t)singles;
    w.ccmc_cum = (long long *)(c->ws + c->L.cc_cum);
    w.st_ccmc = (unsigned long long *)(c->ws + c->L.st_ccmc);
    w.single_key = (uint64_t *)(c->ws + c->L.single_key);
    w.single_pop = (int32_t *)(c->ws + c->L.single_pop);
    w.W = c->W;
    w.hist_len = HIST_LEN;
    c->cur = 0;
    set_main_views(c);

    // tables and per-system device structs
    std::vector<DevSys> ds(c->R);
    std::vector<RepParams> rp(c->R);
    size_t toff = c->L.tables;
    bool put_failed = false;
    auto put = [&](const void *src, size_t bytes) -> const void * {
        if (!bytes) return nullptr;
        char *dst = c->ws + toff;
        if (h2d(c->stream, dst, src, bytes) != hipSuccess) put_failed = true;
        toff += al(bytes);
        return dst;
    };
    for (int r = 0; r < c->R; ++r) {
        const HostSys &s = c->sys[r];
        DevSys &d = ds[r];
        std::memset(&d, 0, sizeof(d));
        d.kind = s.kind;
        d.n_spatial = s.n_spatial;
        d.n_so = s.n_so;
        d.nel = s.nel;
        d.na = s.na;
        d.nb = s.nb;
        d.periodic = s.periodic;
        d.t = s.t;
        d.U = s.U;
        d.u.gmax = s.gmax;
        d.u.gdim = s.gdim;
        d.u.M = s.n_spatial;
        d.u.nel = s.nel;
        if (s.kind == FQ_UEG) {
            // the generator's p_gen = 2 / (C(N,2) n_A) for n_A = M and 2M
            const int64_t npairs = (int64_t)s.nel * (s.nel - 1) / 2;
            d.u.pgen_same = 2.0 / (double)(npairs * s.n_spatial);
            d.u.pgen_opp = 2.0 / (double)(npairs * 2 * s.n_spatial);
        }
        d.vlen = s.vlen;
        d.u.npk = (const int32_t *)put(s.npk.data(), 4 * s.npk.size());
        d.u.vx = (const double *)put(s.vx.data(), 8 * s.vx.size());
        d.u.eps = (const double *)put(s.eps.data(), 8 * s.eps.size());
        d.u.vtab = (const double *)put(s.vtab.data(), 8 * s.vtab.size());
        d.u.grid = (const int16_t *)put(s.grid.data(), 2 * s.grid.size());
        d.h1 = (const double *)put(s.h1.data(), 8 * s.h1.size());
        d.eri = (const double *)put(s.eri.data(), 8 * s.eri.size());
        d.hd = (const double *)put(s.hd.data(), 8 * s.hd.size());
        d.Jt = (const double *)put(s.Jt.data(), 8 * s.Jt.size());
        d.Kt = (const double *)put(s.Kt.data(), 8 * s.Kt.size());
        d.hb_off = (const int64_t *)put(s.hb_off.data(), 8 * s.hb_off.size());
        d.hb_cnt = (const int32_t *)put(s.hb_cnt.data(), 4 * s.hb_cnt.size());
        d.hb_S = (const double *)put(s.hb_S.data(), 8 * s.hb_S.size());
        d.hb_AB = (const uint16_t *)put(s.hb_AB.data(), 2 * s.hb_AB.size());
        d.hb_cdf = (const double *)put(s.hb_cdf.data(), 8 * s.hb_cdf.size());
        std::memcpy(d.ref, s.ref, sizeof(d.ref));
        const fq_qmc &q = qmc[r];
        RepParams &p = rp[r];
        std::memset(&p, 0, sizeof(p));
        p.tau = q.tau;
        p.p_single = q.p_single;
        const double scale = std::ldexp(1.0, q.fixed_point_bits);
        p.cu = q.fixed_point_bits ? (int64_t)std::floor(q.spawn_cutoff * scale + 0.5) : 0;
        p.thr = (int64_t)std::floor(q.initiator_threshold * scale);
        p.k0 = (uint32_t)q.rng_seed;
        p.k1 = (uint32_t)(q.rng_seed >> 32) ^ (uint32_t)q.replica_id;
        p.bits = q.fixed_point_bits;
        p.initiator = q.initiator ? 1 : 0;
        p.sys = r;
    }
    hipError_t he = put_failed ? hipErrorInvalidValue : h2d(c->stream, (void *)w.sys, ds.data(), sizeof(DevSys) * c->R);
    if (he == hipSuccess) he = h2d(c->stream, (void *)w.rep, rp.data(), sizeof(RepParams) * c->R);
    if (he == hipSuccess) he = fill0(c->stream, w.ctl, sizeof(Ctl));
    if (he == hipSuccess) he = fill0(c->stream, c->ws + c->L.st_scan, c->L.main[0][0] - c->L.st_scan);
    if (he == hipSuccess && c->L.single_key > c->L.st_ccmc) he = fill0(c->stream, c->ws + c->L.st_ccmc, c->L.single_key - c->L.st_ccmc);
    if (he == hipSuccess) he = enqueue_setup(0, c->lkind, w, (DevSys *)w.sys, c->R, c->buf[0], 0, nullptr, nullptr, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) { delete c; return FQ_EHIP; }
    c->h00v.resize(c->R);
    for (int r = 0; r < c->R; ++r) {
        DevSys d;
        if (d2h(c->stream, &d, w.sys + r, sizeof(DevSys)) != hipSuccess) { fq_destroy(c); return FQ_EHIP; }
        c->h00v[r] = d.H00;
    }
    if (pinned) {
        he = hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), 0);
        if (he == hipSuccess) he = hipHostMalloc((void **)&c->h_hist, sizeof(EstAcc) * c->R * HIST_LEN, 0);
        if (he == hipSuccess) he = hipHostMalloc((void **)&c->h_shift, 8 * c->R, 0);
        if (he != hipSuccess) { fq_destroy(c); return FQ_EHIP; }
    } else {
        c->h_ctl = new Ctl();
        c->h_hist = new EstAcc[(size_t)c->R * HIST_LEN]();
        c->h_shift = new double[c->R]();
    }

    // grids: persistent tile kernels sized to the resident capacity
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) {
        fq_destroy(c);
        return FQ_EHIP;
    }
    c->grids.scan = ncu * occupancy_blocks(3);
    c->grids.sort = ncu * occupancy_blocks(0);
    c->grids.merge = std::min(ncu * occupancy_blocks(c->W <= 2 ? 1 : 5), PART_MAX_BLOCKS);
    c->grids.reduce = std::min(ncu * occupancy_blocks(2), PART_MAX_BLOCKS);
    c->grids.part = ncu * 4;
    c->grids.spawn = ncu * occupancy_blocks(4);
    // diagonal tables staged in LDS by the single-replica new-determinant kernel
    // tables staged in LDS serve every replica when all replicas share one system
    bool one_system = true;
    for (int r = 1; r < c->R; ++r) one_system = one_system && same_system(sys[0], sys[r]);
    // the LDS-staged table paths of the spawn and diagonal kernels serve determinant keys only
    if (dm_method(c->method)) one_system = false;
    if (one_system && (c->kind == FQ_UEG || c->kind == FQ_MOLECULAR)) {
        const size_t m = (size_t)c->sys[0].n_spatial;
        size_t bytes = c->kind == FQ_UEG ? 8 * (m + m * m) : 8 * (m + 2 * m * m);
        // electron gas on a large basis: kinetic energies, v by |dn|^2, packed momenta
        if (c->kind == FQ_UEG && bytes > (size_t)ND_LDS_MAX) bytes = 8 * m + 8 * (size_t)c->sys[0].vlen + 4 * m;
        if (bytes <= (size_t)ND_LDS_MAX) w.lds_diag = (int32_t)bytes;
    }
    // heat-bath pair weights (upper triangle) staged in LDS by the single-replica spawn kernel
    if (one_system && c->kind == FQ_MOLECULAR) {
        const size_t nso = (size_t)c->sys[0].n_so;
        const size_t bytes = 8 * (nso * (nso - 1) / 2);
        if (bytes <= 32768) {
            c->grids.spawn_lds = (int)bytes;
            w.lds_tables = (int32_t)bytes;
        }
    }
    // UEG generator tables staged in LDS by the single-replica spawn kernel
    if (one_system && c->kind == FQ_UEG) {
        const HostSys &s0 = c->sys[0];
        const size_t bytes = ((4 * (size_t)s0.n_spatial + 15) & ~(size_t)15) + ((8 * (size_t)s0.vlen + 15) & ~(size_t)15) +
                             2 * s0.grid.size();
        if (bytes <= 32768) {
            c->grids.spawn_lds = (int)bytes;
            w.lds_tables = (int32_t)bytes;
        }
    }
    c->grids.hist = ncu * 4;
    c->grids.fixup = ncu * 2;
    c->grids.det = ncu * 4;
    c->grids.newdiag = ncu * 8;

    c->shift.assign(c->R, 0.0);
    c->vary.assign(c->R, 0);
    c->rs_max.assign(c->R, 0.0);
    c->nprev.assign(c->R, 0);
    c->last.resize(c->R);
    c->hist.assign(c->R, {});
    // initial list: the reference of each replica
    std::vector<HostEntry> init(c->R);
    for (int r = 0; r < c->R; ++r) {
        HostEntry &e = init[r];
        std::memset(&e, 0, sizeof(e));
        std::memcpy(e.key, c->sys[r].ref, sizeof(e.key));
        if (dm_method(c->method)) e.key[1] = c->sys[r].ref[0];  // the pair (D_0, D_0)
        e.skey = host_skey(host_hash(e.key, c->W) & c->hmask, (uint32_t)r, c->rb);
        const double scale = std::ldexp(1.0, qmc[r].fixed_point_bits);
        const double u = std::floor(qmc[r].init_pop * scale + 0.5);
        if (u > 2147483647.0) { fq_destroy(c); return FQ_EOVERFLOW; }
        e.pop = (int32_t)u;
        e.dslot = -1;
        c->shift[r] = qmc[r].initial_shift;
    }
    std::vector<HostEntry> nz;
    for (auto &e : init)
        if (e.pop != 0) nz.push_back(e);
    std::sort(nz.begin(), nz.end(), [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, c->W); });
    for (int r = 0; r < c->R; ++r) c->h_shift[r] = c->shift[r];
    if (h2d(c->stream, w.shift, c->h_shift, 8 * c->R) != hipSuccess) { fq_destroy(c); return FQ_EHIP; }
    if (upload_main(c, nz) != FQ_OK || host_estimators(c) != FQ_OK) { fq_destroy(c); return FQ_EHIP; }
    c->static_dev = static_dev;  // from here on fq_destroy gives the static array back
    *out = c;
    return FQ_OK;
}

// ---------------------------------------------------------------------------
// Static device workspace of fq_init_system_static: one array per device
// (each device that loads the library holds it until the process ends). Host
// code never passes `scratch` itself to the device (the name is a host-side
// stand-in); it passes the device address that hipGetSymbolAddress returns for
// the current device, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FQ_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[MAX_DEVICES] = {nullptr};  // device address of scratch, per device
bool g_static_busy[MAX_DEVICES] = {false};    // a live context holds the device's array

// reserves the current device's array; *dev receives the device index
fq_status static_workspace_acquire(void **ptr, int *dev)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= MAX_DEVICES) return FQ_EHIP;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[d]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FQ_EHIP;
        g_static_ptr[d] = p;
    }
    if (g_static_busy[d]) return FQ_ESTATE;
    g_static_busy[d] = true;
    *ptr = g_static_ptr[d];
    *dev = d;
    return FQ_OK;
}

void static_workspace_release(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[dev] = false;
}

}  // namespace

extern "C" {

fq_status fq_init_system(fq_ctx **out, const fq_system *sys, const fq_qmc *qmc, const fq_semistoch *ss,
                         int32_t n_instances, int64_t main_capacity, int64_t spawn_capacity, void *d_workspace,
                         size_t ws_bytes, void *hip_stream)
{
    return init_system(out, sys, qmc, ss, n_instances, main_capacity, spawn_capacity, d_workspace, ws_bytes,
                       hip_stream, true, -1);
}

fq_status fq_init_system_static(fq_ctx **out, const fq_system *sys, const fq_qmc *qmc, const fq_semistoch *ss,
                                int32_t n_instances, int64_t main_capacity, int64_t spawn_capacity,
                                void *hip_stream)
{
    if (!out) return FQ_EINVAL;
    *out = nullptr;
    const size_t need = fq_workspace_bytes(sys, qmc, ss, n_instances, main_capacity, spawn_capacity);
    if (need == 0) return FQ_EINVAL;
    if (need > (size_t)FQ_STATIC_WORKSPACE_BYTES) return FQ_ECAPACITY;
    void *ptr = nullptr;
    int dev = -1;
    const fq_status st = static_workspace_acquire(&ptr, &dev);
    if (st != FQ_OK) return st;
    const fq_status r = init_system(out, sys, qmc, ss, n_instances, main_capacity, spawn_capacity, ptr,
                                    (size_t)FQ_STATIC_WORKSPACE_BYTES, hip_stream, false, dev);
    // a failed set-up has freed its context, which never held the array
    if (r != FQ_OK) static_workspace_release(dev);
    return r;
}

fq_status fq_step(fq_ctx *c, int32_t n_iterations)
{
    if (!c) return FQ_EINVAL;
    if (n_iterations < 0) return fail(c, FQ_EINVAL, "negative iteration count");
    const int A = c->qmc[0].shift_period;
    for (int r = 0; r < c->R; ++r) c->hist[r].clear();
    std::fill(c->stage_ms, c->stage_ms + 7, 0.0);
    std::fill(c->kernel_ms, c->kernel_ms + N_KERNEL_SLOTS, 0.0);
    c->timed_iterations = 0;
    c->iter_ms.clear();
    constexpr int NE = N_KERNEL_SLOTS + 1;
    std::vector<hipEvent_t> evs;
    int done = 0;
    while (done < n_iterations) {
        // CCMC: the prefix of |N_i| travels in look-back words of 38 bits; a
        // block of iterations starts only with room for its growth
        if (c->method == FQ_CCMC && c->last[0].n_walkers_units >= (int64_t(1) << 36))
            return fail(c, FQ_EOVERFLOW, "CCMC: the excip population exceeds 2^36 units");
        // iterations until the next host decision point (shift update, D selection, end)
        int64_t stop = c->t + (n_iterations - done);
        const int64_t next_shift = (c->t / A + 1) * A;
        stop = std::min(stop, next_shift);
        if (c->has_ss && !c->ss_active && c->t < c->ss.start_iteration) stop = std::min<int64_t>(stop, c->ss.start_iteration);
        stop = std::min<int64_t>(stop, c->t + HIST_LEN / 2);
        // The look-back status words carry the iteration counter modulo
        // 2^20. A block never crosses a multiple of 2^20, and before the first
        // iteration of each such period every status array is cleared, so no
        // word written 2^20 iterations earlier can carry a matching epoch.
        constexpr int64_t EPOCH_PERIOD = int64_t(1) << 20;
        stop = std::min<int64_t>(stop, ((c->t + 1) / EPOCH_PERIOD + 1) * EPOCH_PERIOD - 1);
        if ((c->t + 1) % EPOCH_PERIOD == 0) {
            HIPCHK(c, fill0(c->stream, c->ws + c->L.st_scan, c->L.part_red - c->L.st_scan));
            if (c->L.single_key > c->L.st_ccmc)
                HIPCHK(c, fill0(c->stream, c->ws + c->L.st_ccmc, c->L.single_key - c->L.st_ccmc));
        }
        const int64_t t0 = c->t;
        const int cur0 = c->cur;
        const int nb = (int)(stop - t0);
        if (c->timing) {
            evs.resize((size_t)nb * NE);
            for (auto &e : evs) (void)hipEventCreate(&e);
        }
        const bool use_graph = c->graph && !c->timing && nb == A;
        if (use_graph) {
            // one captured block of A iterations per main-list parity, replayed
            const int b = c->cur;
            if (!c->gexec[b] || c->graph_len[b] != nb) {
                if (c->gexec[b]) (void)hipGraphExecDestroy(c->gexec[b]);
                if (c->graphs[b]) (void)hipGraphDestroy(c->graphs[b]);
                c->gexec[b] = nullptr;
                c->graphs[b] = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < nb; ++k) {
                    hipError_t he = enqueue_iteration(c->w, c->lkind, c->grids, c->stream, nullptr);
                    if (he != hipSuccess) {
                        hipGraph_t junk;
                        (void)hipStreamEndCapture(c->stream, &junk);
                        if (junk) (void)hipGraphDestroy(junk);
                        return fail(c, FQ_EHIP, std::string("capture: ") + hipGetErrorString(he));
                    }
                    c->cur ^= 1;
                    set_main_views(c);
                }
                HIPCHK(c, hipStreamEndCapture(c->stream, &c->graphs[b]));
                HIPCHK(c, hipGraphInstantiate(&c->gexec[b], c->graphs[b], nullptr, nullptr, 0));
                c->graph_len[b] = nb;
                c->cur = b;
                set_main_views(c);
            }
            HIPCHK(c, hipGraphLaunch(c->gexec[b], c->stream));
            c->cur = b ^ (nb & 1);
            set_main_views(c);
        } else {
            for (int k = 0; k < nb; ++k) {
                hipError_t he = enqueue_iteration(c->w, c->lkind, c->grids, c->stream, c->timing ? &evs[(size_t)k * NE] : nullptr);
                if (he != hipSuccess) return fail(c, FQ_EHIP, std::string("launch: ") + hipGetErrorString(he));
                c->cur ^= 1;
                set_main_views(c);
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->h_ctl, c->w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->h_hist, c->w.hist, sizeof(EstAcc) * c->R * HIST_LEN, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->timing) {
            // stage boundaries in the launch order: scan+partition, spawn, sort
            // (histogram + 8 passes), reduce (2 passes + fix-up), projection, merge
            static const int stage_of[N_KERNEL_SLOTS] = {0, 0, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 5, 5, 5, 4, 4, 4, 4, 4};
            for (int k = 0; k < nb; ++k) {
                hipEvent_t *e = &evs[(size_t)k * NE];
                float ms = 0.f;
                for (int q = 0; q < N_KERNEL_SLOTS; ++q) {
                    (void)hipEventElapsedTime(&ms, e[q], e[q + 1]);
                    c->kernel_ms[q] += ms;
                    c->stage_ms[stage_of[q]] += ms;
                }
                (void)hipEventElapsedTime(&ms, e[0], e[N_KERNEL_SLOTS]);
                c->stage_ms[6] += ms;
                c->iter_ms.push_back(ms);
            }
            c->timed_iterations += nb;
            for (auto &e : evs) (void)hipEventDestroy(e);
            evs.clear();
        }
        const Ctl &ctl = *c->h_ctl;
        if (!ctl.err && (int64_t)ctl.t != stop)
            return fail(c, FQ_ESTATE, "device iteration counter " + std::to_string(ctl.t) + " after a block ending at " +
                                          std::to_string(stop));
        if (ctl.err) {
            // ctl is the pinned host copy of the device counters, which the
            // restore below overwrites: keep the error bits
            const uint32_t err = ctl.err;
            const int64_t tf = ctl.t;  // failing iteration
            c->cur = cur0 ^ (int)((tf - 1 - t0) & 1);
            set_main_views(c);
            // restore the device counters to the start of the failing iteration
            Ctl fix = ctl;
            fix.err = 0;
            fix.t = (uint32_t)(tf - 1);
            fix.n_main_new = ctl.n_main;
            HIPCHK(c, h2d(c->stream, c->w.ctl, &fix, sizeof(Ctl)));
            // the failing merge may have written attempt offsets and deterministic
            // positions for a list that is discarded: rebuild them for the restored one
            {
                std::vector<HostEntry> e;
                int64_t nres;
                fq_status st2 = download_main(c, e, nres);
                if (st2) return st2;
                st2 = upload_main(c, e);
                if (st2) return st2;
                if (c->ss_active) {
                    std::vector<int32_t> pos((size_t)c->D * c->R, 0);
                    for (int64_t i = 0; i < nres; ++i)
                        if (e[i].dslot >= 0) {
                            const uint32_t rep = c->rb ? (uint32_t)(e[i].skey >> (64 - c->rb)) : 0u;
                            pos[(size_t)rep * c->D + e[i].dslot] = (int32_t)i;
                        }
                    HIPCHK(c, h2d(c->stream, c->ws + c->L.ds[3], pos.data(), 4 * pos.size()));
                }
            }
            fold_spawn_ratio(c, t0 + 1, tf - 1);
            for (int64_t it = t0 + 1; it < tf; ++it)
                for (int r = 0; r < c->R; ++r) {
                    fq_estimators_t e;
                    estimators_from_acc(c, r, c->h_hist[(size_t)(it % HIST_LEN) * c->R + r], e);
                    e.shift = c->shift[r];
                    e.vary_shift = c->vary[r];
                    c->hist[r].push_back(e);
                    c->last[r] = e;
                }
            c->t = tf - 1;
            if (err & (ERR_OVERFLOW | ERR_ATTEMPTS)) return fail(c, FQ_EOVERFLOW, "population or spawn exceeds the fixed-point range");
            if (err & ERR_COLLISION) return fail(c, FQ_ESTATE, "more than 64 spawned determinants share one sort key (not a hash collision)");
            if (err & ERR_NOREF) return fail(c, FQ_ENOREF, "CCMC: the reference determinant holds no walkers");
            if (err & ERR_SPAWN_CAP) return fail(c, FQ_ECAPACITY, "spawn capacity exceeded");
            return fail(c, FQ_ECAPACITY, "main list capacity exceeded");
        }
        fold_spawn_ratio(c, t0 + 1, stop);
        for (int64_t it = t0 + 1; it <= stop; ++it) {
            for (int r = 0; r < c->R; ++r) {
                fq_estimators_t e;
                estimators_from_acc(c, r, c->h_hist[(size_t)(it % HIST_LEN) * c->R + r], e);
                if (it % A == 0) {
                    const double target = c->qmc[r].target_population * std::ldexp(1.0, c->qmc[r].fixed_point_bits);
                    const int64_t nw = e.n_walkers_units;
                    if (!c->vary[r]) {
                        if ((double)nw >= target) {
                            c->vary[r] = 1;
                            c->nprev[r] = nw;
                        }
                    } else {
                        const double cc = c->qmc[r].shift_damping / ((double)A * c->qmc[r].tau);
                        const double ratio = (double)nw / (double)c->nprev[r];
                        c->shift[r] = c->shift[r] - cc * std::log(ratio);
                        c->nprev[r] = nw;
                    }
                    // time-step search (the tutorial's tau_search), after the shift
                    // update: tau only decreases, so that tau |H_ji| / p_gen <= 1 for
                    // every attempt so far and tau (K_ii - S) <= 1 for the entries of
                    // the last death step (the block's last iteration is this one)
                    if (c->qmc[r].tau_search && it == stop) {
                        double tau = c->qmc[r].tau;
                        if (c->rs_max[r] > 0.0) {
                            const double bnd = 1.0 / c->rs_max[r];
                            if (bnd < tau) tau = bnd;
                        }
                        const unsigned long long kd = c->h_hist[(size_t)(stop % HIST_LEN) * c->R + r].kd_key;
                        if (kd != 0) {
                            const double d = from_ordered_key(kd) - c->shift[r];
                            if (d > 0.0) {
                                const double bnd = 1.0 / d;
                                if (bnd < tau) tau = bnd;
                            }
                        }
                        if (tau != c->qmc[r].tau) {
                            c->qmc[r].tau = tau;
                            HIPCHK(c, h2d(c->stream, (char *)c->w.rep + (size_t)r * sizeof(RepParams) + offsetof(RepParams, tau),
                                          &c->qmc[r].tau, sizeof(double)));
                        }
                    }
                }
                e.tau = c->qmc[r].tau;
                e.shift = c->shift[r];
                e.vary_shift = c->vary[r];
                c->hist[r].push_back(e);
                c->last[r] = e;
            }
        }
        c->t = stop;
        done += nb;
        for (int r = 0; r < c->R; ++r) c->h_shift[r] = c->shift[r];
        HIPCHK(c, hipMemcpyAsync(c->w.shift, c->h_shift, 8 * c->R, hipMemcpyHostToDevice, c->stream));
        if (c->has_ss && !c->ss_active && c->t >= c->ss.start_iteration) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            fq_status st = select_detspace(c);
            if (st) return st;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FQ_OK;
}

fq_status fq_estimators(const fq_ctx *c, int32_t instance, fq_estimators_t *out)
{
    if (!c || !out || instance < 0 || instance >= c->R) return FQ_EINVAL;
    *out = c->last[instance];
    return FQ_OK;
}

fq_status fq_estimator_history(const fq_ctx *c, int32_t instance, fq_estimators_t *out, int32_t cap, int32_t *n_out)
{
    if (!c || !out || !n_out || instance < 0 || instance >= c->R || cap < 0) return FQ_EINVAL;
    const auto &h = c->hist[instance];
    const int n = (int)std::min<size_t>(h.size(), (size_t)cap);
    for (int i = 0; i < n; ++i) out[i] = h[h.size() - n + i];
    *n_out = n;
    return FQ_OK;
}

// [lo, hi) of one instance in the current main list: the replica id is the
// most significant field of the sort key, so each instance is one contiguous
// run, found by binary search over the device array
fq_status instance_range(fq_ctx *c, int instance, int64_t &lo, int64_t &hi)
{
    HIPCHK(c, d2h(c->stream, c->h_ctl, c->w.ctl, sizeof(Ctl)));
    const int64_t n = c->h_ctl->n_main_new;
    if (c->rb == 0) {
        lo = 0;
        hi = n;
        return FQ_OK;
    }
    const uint64_t *sk = c->buf[c->cur].skey;
    auto first_rep_at_least = [&](uint64_t r, int64_t &pos) -> fq_status {
        int64_t a = 0, b = n;
        while (a < b) {
            const int64_t m = a + (b - a) / 2;
            uint64_t v;
            HIPCHK(c, d2h(c->stream, &v, sk + m, 8));
            if ((v >> (64 - c->rb)) < r) a = m + 1;
            else b = m;
        }
        pos = a;
        return FQ_OK;
    };
    fq_status st = first_rep_at_least((uint64_t)instance, lo);
    if (st) return st;
    return first_rep_at_least((uint64_t)instance + 1, hi);
}

}  // extern "C"

namespace {

// word-major keys kk[q * n + i] and populations, written out in key order
template <int W>
void sort_rows(const std::vector<uint64_t> &kk, const std::vector<int32_t> &pp, int64_t n, uint64_t *keys,
               int32_t *pops)
{
    struct Row {
        uint64_t k[W];
        int32_t pop;
    };
    std::vector<Row> rows(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < W; ++q) rows[i].k[q] = kk[(size_t)q * n + i];
        rows[i].pop = pp[i];
    }
    std::sort(rows.begin(), rows.end(), [](const Row &a, const Row &b) {
        for (int q = W - 1; q >= 0; --q)
            if (a.k[q] != b.k[q]) return a.k[q] < b.k[q];
        return false;
    });
    for (int64_t i = 0; i < n; ++i) {
        if (keys)
            for (int q = 0; q < W; ++q) keys[(size_t)i * W + q] = rows[i].k[q];
        if (pops) pops[i] = rows[i].pop;
    }
}

}  // namespace

extern "C" {

fq_status fq_export_walkers(const fq_ctx *cc, int32_t instance, uint64_t *keys, int32_t *pops, int64_t cap,
                            int64_t *n_out)
{
    fq_ctx *c = const_cast<fq_ctx *>(cc);
    if (!c || instance < 0 || instance >= c->R || !n_out) return FQ_EINVAL;
    int64_t lo, hi;
    fq_status st = instance_range(c, instance, lo, hi);
    if (st) return st;
    const int64_t n = hi - lo;
    const int W = c->W;
    *n_out = n;
    if (n > cap) return fail(c, FQ_ECAPACITY, "export buffer too small");
    if (!keys && !pops) return FQ_OK;
    const MainList &m = c->buf[c->cur];
    std::vector<uint64_t> kk((size_t)n * W);
    std::vector<int32_t> pp(n);
    if (n) {
        for (int q = 0; q < W; ++q)
            HIPCHK(c, d2h(c->stream, kk.data() + (size_t)q * n, m.key + (size_t)q * c->main_cap + lo, 8 * n));
        HIPCHK(c, d2h(c->stream, pp.data(), m.pop + lo, 4 * n));
    }
    // key order (most significant word first): rows of (key words, population)
    // sorted in place, so that every comparison reads one contiguous row
    switch (W) {
    case 1: sort_rows<1>(kk, pp, n, keys, pops); break;
    case 2: sort_rows<2>(kk, pp, n, keys, pops); break;
    case 4: sort_rows<4>(kk, pp, n, keys, pops); break;
    default: sort_rows<8>(kk, pp, n, keys, pops); break;
    }
    return FQ_OK;
}

fq_status fq_import_walkers(fq_ctx *c, int32_t instance, const uint64_t *keys, const int32_t *pops, int64_t n,
                            double shift, int64_t iteration, int32_t vary_shift, int64_t n_prev)
{
    if (!c || instance < 0 || instance >= c->R || n < 0 || (n > 0 && (!keys || !pops)) || iteration < 0)
        return FQ_EINVAL;
    std::vector<HostEntry> e;
    int64_t m;
    fq_status st = download_main(c, e, m);
    if (st) return st;
    std::vector<HostEntry> out;
    for (const HostEntry &x : e) {
        const uint32_t rep = c->rb ? (uint32_t)(x.skey >> (64 - c->rb)) : 0u;
        if ((int)rep != instance) out.push_back(x);
    }
    std::vector<HostEntry> add;
    for (int64_t i = 0; i < n; ++i) {
        if (pops[i] == 0) continue;
        HostEntry x;
        std::memset(&x, 0, sizeof(x));
        for (int q = 0; q < c->W; ++q) x.key[q] = keys[(size_t)i * c->W + q];
        if (c->method == FQ_CCMC) {
            // CCMC: no amplitude beyond the truncation level
            int d = 0;
            for (int q = 0; q < c->W; ++q) d += __builtin_popcountll(x.key[q] ^ c->sys[instance].ref[q]);
            if (d / 2 > c->qmc[0].ccmc_truncation) return fail(c, FQ_EINVAL, "excitor beyond the truncation level");
        }
        x.skey = host_skey(host_hash(x.key, c->W) & c->hmask, (uint32_t)instance, c->rb);
        x.pop = pops[i];
        x.dslot = -1;
        add.push_back(x);
    }
    std::sort(add.begin(), add.end(), [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, c->W); });
    for (size_t i = 1; i < add.size(); ++i)
        if (add[i].skey == add[i - 1].skey && key_cmp_host(add[i].key, add[i - 1].key, c->W) == 0)
            return fail(c, FQ_EINVAL, "duplicate determinant in import");
    out.insert(out.end(), add.begin(), add.end());
    for (auto &x : out) x.dslot = -1;
    std::sort(out.begin(), out.end(), [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, c->W); });
    c->shift[instance] = shift;
    c->vary[instance] = vary_shift;
    c->nprev[instance] = n_prev;
    c->t = iteration;
    Ctl ctl;
    HIPCHK(c, d2h(c->stream, &ctl, c->w.ctl, sizeof(Ctl)));
    ctl.t = (uint32_t)iteration;
    ctl.err = 0;
    ctl.ss_active = 0;
    HIPCHK(c, h2d(c->stream, c->w.ctl, &ctl, sizeof(Ctl)));
    c->ss_active = false;
    for (int r = 0; r < c->R; ++r) c->h_shift[r] = c->shift[r];
    HIPCHK(c, h2d(c->stream, c->w.shift, c->h_shift, 8 * c->R));
    st = upload_main(c, out);
    if (st) return st;
    st = host_estimators(c);
    if (st) return st;
    if (c->has_ss && c->t >= c->ss.start_iteration) return select_detspace(c);
    return FQ_OK;
}

fq_status fq_export_spawns(const fq_ctx *cc, int32_t instance, uint64_t *keys, int32_t *amps, uint8_t *init,
                           int64_t cap, int64_t *n_out)
{
    fq_ctx *c = const_cast<fq_ctx *>(cc);
    if (!c || instance < 0 || instance >= c->R || !n_out) return FQ_EINVAL;
    Ctl ctl;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, d2h(c->stream, &ctl, c->w.ctl, sizeof(Ctl)));
    const int64_t n = (int64_t)std::min<unsigned long long>(ctl.n_spawn, (unsigned long long)c->spawn_cap);
    std::vector<uint64_t> sk(n), kk((size_t)n * c->W);
    std::vector<uint32_t> ix(n);
    std::vector<int32_t> am(n);
    std::vector<uint8_t> in(n);
    if (n) {
        HIPCHK(c, d2h(c->stream, sk.data(), c->w.sp.skey, 8 * n));
        HIPCHK(c, d2h(c->stream, ix.data(), c->w.sp.idx, 4 * n));
        std::vector<uint64_t> rec((size_t)n * (c->W + 1));
        HIPCHK(c, d2h(c->stream, rec.data(), c->w.sp.rec, 8 * rec.size()));
        for (int64_t j = 0; j < n; ++j) {
            for (int q = 0; q < c->W; ++q) kk[(size_t)q * n + j] = rec[(size_t)j * (c->W + 1) + q];
            const uint64_t ai = rec[(size_t)j * (c->W + 1) + c->W];
            am[j] = (int32_t)(uint32_t)ai;
            in[j] = (uint8_t)(ai >> 32);
        }
    }
    int64_t o = 0;
    for (int64_t p = 0; p < n; ++p) {
        const uint32_t rep = c->rb ? (uint32_t)(sk[p] >> (64 - c->rb)) : 0u;
        if ((int)rep != instance) continue;
        const uint32_t j = ix[p];
        if (o < cap) {
            if (keys)
                for (int q = 0; q < c->W; ++q) keys[(size_t)o * c->W + q] = kk[(size_t)q * n + j];
            if (amps) amps[o] = am[j];
            if (init) init[o] = in[j];
        }
        ++o;
    }
    *n_out = o;
    return o > cap ? fail(c, FQ_ECAPACITY, "export buffer too small") : FQ_OK;
}

fq_status fq_detspace(const fq_ctx *cc, int32_t instance, uint64_t *keys, double *last_y, int64_t cap, int64_t *n_out)
{
    fq_ctx *c = const_cast<fq_ctx *>(cc);
    if (!c || instance < 0 || instance >= c->R || !n_out) return FQ_EINVAL;
    if (!c->ss_active) {
        *n_out = 0;
        return FQ_OK;
    }
    *n_out = c->D;
    if (cap < c->D) return fail(c, FQ_ECAPACITY, "buffer too small");
    if (keys) std::memcpy(keys, c->dkeys[instance].data(), 8 * (size_t)c->D * c->W);
    if (last_y) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, d2h(c->stream, last_y, c->w.ds.y + (size_t)instance * c->D, 8 * (size_t)c->D));
    }
    return FQ_OK;
}

fq_status fq_info(const fq_ctx *c, int32_t *W, int32_t *n_so, double *e_ref)
{
    if (!c) return FQ_EINVAL;
    if (W) *W = c->W;
    if (n_so) *n_so = c->sys[0].n_so;
    if (e_ref) *e_ref = c->h00v[0];
    return FQ_OK;
}

fq_status fq_set_timing(fq_ctx *c, int32_t on)
{
    if (!c) return FQ_EINVAL;
    c->timing = on != 0;
    return FQ_OK;
}

fq_status fq_stage_times(const fq_ctx *c, double *ms7)
{
    if (!c || !ms7) return FQ_EINVAL;
    std::memcpy(ms7, c->stage_ms, sizeof(c->stage_ms));
    return FQ_OK;
}

fq_status fq_shift_state(const fq_ctx *c, int32_t instance, double *shift, int64_t *n_prev, int32_t *vary_shift)
{
    if (!c || instance < 0 || instance >= c->R) return FQ_EINVAL;
    if (shift) *shift = c->shift[instance];
    if (n_prev) *n_prev = c->nprev[instance];
    if (vary_shift) *vary_shift = c->vary[instance];
    return FQ_OK;
}

fq_status fq_iteration_times(const fq_ctx *c, double *ms, int64_t cap, int64_t *n_out)
{
    if (!c || !n_out || (cap > 0 && !ms)) return FQ_EINVAL;
    const int64_t n = std::min<int64_t>(cap, (int64_t)c->iter_ms.size());
    for (int64_t i = 0; i < n; ++i) ms[i] = c->iter_ms[i];
    *n_out = n;
    return FQ_OK;
}

fq_status fq_set_graph(fq_ctx *c, int32_t on)
{
    if (!c) return FQ_EINVAL;
    if (on && (c->stream == nullptr || c->stream == hipStreamLegacy))
        return fail(c, FQ_EINVAL, "graph replay needs a stream other than the legacy default stream");
    c->graph = on != 0;
    if (!c->graph) drop_graphs(c);
    return FQ_OK;
}

fq_status fq_set_sort_key_bits(fq_ctx *c, int32_t bits)
{
    if (!c) return FQ_EINVAL;
    if (bits < 1 || bits > 64) return fail(c, FQ_EINVAL, "sort-key hash bits must lie in 1..64");
    if (c->R < 2)
        return fail(c, FQ_EINVAL, "sort-key truncation needs two or more instances (a single instance's kernels use the "
                                  "sort key as the determinant's hash)");
    if (c->ss_active) return fail(c, FQ_ESTATE, "sort-key truncation must precede the deterministic space");
    c->hmask = bits == 64 ? ~0ull : ~((1ull << (64 - bits)) - 1);
    c->w.hmask = c->hmask;
    // the current list in the order of the new sort keys (upload_main drops
    // the captured graphs, whose kernel arguments hold the old mask)
    std::vector<HostEntry> e;
    int64_t n = 0;
    fq_status st = download_main(c, e, n);
    if (st != FQ_OK) return st;
    for (auto &x : e) {
        const uint32_t rep = c->rb ? (uint32_t)(x.skey >> (64 - c->rb)) : 0u;
        x.skey = host_skey(host_hash(x.key, c->W) & c->hmask, rep, c->rb);
    }
    std::sort(e.begin(), e.end(), [&](const HostEntry &a, const HostEntry &b) { return entry_less(a, b, c->W); });
    return upload_main(c, e);
}

fq_status fq_set_launch(fq_ctx *c, const int32_t *blocks, int32_t n)
{
    if (!c || !blocks || n < 0) return FQ_EINVAL;
    int *dst[5] = {&c->grids.spawn, &c->grids.merge, &c->grids.sort, &c->grids.reduce, &c->grids.newdiag};
    // the merge and the reduction keep one row of estimator partials per block
    const int cap[5] = {1 << 20, PART_MAX_BLOCKS, 1 << 20, PART_MAX_BLOCKS, 1 << 20};
    for (int i = 0; i < n && i < 5; ++i)
        if (blocks[i] > cap[i]) return fail(c, FQ_EINVAL, "launch geometry out of range");
    for (int i = 0; i < n && i < 5; ++i)
        if (blocks[i] > 0) *dst[i] = blocks[i];
    drop_graphs(c);
    return FQ_OK;
}

fq_status fq_set_tiles(fq_ctx *c, const int32_t *tiles, int32_t n)
{
    if (!c || !tiles || n < 0) return FQ_EINVAL;
    int *dst[3] = {&c->grids.spawn_i, &c->grids.merge_i, &c->grids.sort_i};
    const int ok[3][3] = {{2, 4, 8}, {1, 2, 4}, {8, 12, 16}};
    for (int i = 0; i < n && i < 3; ++i)
        if (tiles[i] > 0 && tiles[i] != ok[i][0] && tiles[i] != ok[i][1] && tiles[i] != ok[i][2])
            return fail(c, FQ_EINVAL, "tile shape not among the compiled variants");
    for (int i = 0; i < n && i < 3; ++i)
        if (tiles[i] > 0) *dst[i] = tiles[i];
    drop_graphs(c);
    return FQ_OK;
}

fq_status fq_get_tiles(const fq_ctx *c, int32_t *tiles, int32_t n)
{
    if (!c || !tiles || n < 0) return FQ_EINVAL;
    const int src[3] = {c->grids.spawn_i, c->grids.merge_i, c->grids.sort_i};
    for (int i = 0; i < n && i < 3; ++i) tiles[i] = src[i];
    return FQ_OK;
}

fq_status fq_get_launch(const fq_ctx *c, int32_t *blocks, int32_t n)
{
    if (!c || !blocks || n < 0) return FQ_EINVAL;
    const int src[5] = {c->grids.spawn, c->grids.merge, c->grids.sort, c->grids.reduce, c->grids.newdiag};
    for (int i = 0; i < n && i < 5; ++i) blocks[i] = src[i];
    return FQ_OK;
}

fq_status fq_kernel_times(const fq_ctx *c, double *ms, int32_t cap, int32_t *n_slots, int64_t *n_iterations)
{
    if (!c || (!ms && cap > 0)) return FQ_EINVAL;
    for (int q = 0; q < cap && q < N_KERNEL_SLOTS; ++q) ms[q] = c->kernel_ms[q];
    if (n_slots) *n_slots = N_KERNEL_SLOTS;
    if (n_iterations) *n_iterations = c->timed_iterations;
    return FQ_OK;
}

const char *fq_last_error(const fq_ctx *c) { return c ? c->err.c_str() : "null context"; }

void fq_destroy(fq_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->pinned) {
        if (c->h_ctl) (void)hipHostFree(c->h_ctl);
        if (c->h_hist) (void)hipHostFree(c->h_hist);
        if (c->h_shift) (void)hipHostFree(c->h_shift);
    } else {
        delete c->h_ctl;
        delete[] c->h_hist;
        delete[] c->h_shift;
    }
    if (c->static_dev >= 0) static_workspace_release(c->static_dev);
    delete c;
}

}  // extern "C"
