// Kernels of one FCIQMC projector iteration on gfx950 (declarations shared by
// the kernel and host translation units).
#pragma once

#include "fq_device.h"

namespace fq {

// Per-replica run parameters (device copy).
struct RepParams {
    double tau;
    double p_single;
    int64_t cu;        // spawn cutoff in units (real mode)
    int64_t thr;       // initiator threshold in units (strict >)
    uint32_t k0, k1;   // Philox key
    int32_t bits;      // fixed-point bits b
    int32_t initiator;
    int32_t sys;       // index of this replica's DevSys
    int32_t pad;
};

// Error bits raised on the device; once any bit is set every later kernel
// returns immediately, so the lists of the failing iteration's input survive.
enum : uint32_t {
    ERR_SPAWN_CAP = 1u,
    ERR_MAIN_CAP = 2u,
    ERR_OVERFLOW = 4u,
    ERR_ATTEMPTS = 8u,
    ERR_UNIQ_CAP = 16u,
    ERR_COLLISION = 32u,
    ERR_NOREF = 64u,  // CCMC: the reference holds no walkers (cluster weights divide by N_0)
};

enum : int {
    TK_SCAN = 0,
    TK_SORT = 1,   // 8 passes: 1..8
    TK_RED1 = 9,
    TK_RED2 = 10,
    TK_MERGE = 11,
    TK_SPAWN = 12,
    TK_CCMC = 13,
    TK_COUNT = 16,
};

struct Ctl {
    long long n_main;      // determinants in the current main list (all replicas)
    long long n_main_new;  // written by the merge
    long long n_att;       // total spawning attempts this iteration
    long long n_att_new;   // attempts of the list the merge has just written
    unsigned long long n_spawn;  // spawned walkers written
    long long n_uniq;      // distinct spawned determinants
    uint32_t t;            // iteration counter (1 = first iteration)
    uint32_t err;
    uint32_t collision;    // equal sort keys with different determinants seen
    uint32_t ss_active;
    uint32_t pad_ts;
    uint32_t tickets[TK_COUNT];
    uint32_t hist[8][256];  // radix-sort digit histogram of the spawned keys
    // CCMC: N_0 and the sum of |N_i| over the excitors at the start of the
    // iteration, and the singles of the new list queued for the estimator
    long long ccmc_n0;
    long long ccmc_nex;
    uint32_t n_single;
    uint32_t pad_ccmc;
};

// Per-replica estimator accumulators (exact integers).
struct EstAcc {
    long long nw, nocc, n0, nspawn, nuniq, flips, rej_units, death_sum, spawn_sum, rej_sum;
    long long limbs[4];
    long long t;
    long long ccmc_rec;  // CCMC: records written by the composite clusters this iteration
    double ss_err;  // split projection: max relative error of the last check
    // CCMC: exact limbs (2^-64) of sum over pairs of singles a < b of
    // H_0,ab sgn(a_a a_b D_0) N_a N_b
    long long pair[4];
    // time-step search, this iteration: bits of the largest |H_ji| / p_gen of
    // the replica's attempts (a non-negative double orders as its bits) and
    // the order-preserving key of the largest K_ii of its death step (0: none)
    unsigned long long rs_bits;
    unsigned long long kd_key;
};
constexpr int EST_FIELDS = 14;
// replicas whose estimator partials a block keeps in LDS (the rest are added
// to global memory directly), and the largest grid of the kernels that write
// partials
constexpr int ACC_LDS_R = 64;
// keys per radix-sort tile: 256 threads x sort_items, sort_items in {8, 12, 16}
// chosen per context (the host sizes the per-tile digit status words for the
// smallest tile)
constexpr int SORT_TILE_MIN = 2048;

// spawn tiles: SP_T threads of SI attempts each (2, 4 or 8 for keys of up to
// two words, chosen per context; 2 for longer keys, whose children take more
// registers); the attempt partition is sized for the smallest tile
constexpr int SP_T = 256;
constexpr int SPAN_MIN = 2 * SP_T;
constexpr int PART_MAX_BLOCKS = 8192;
// largest diagonal-table staging of the new-determinant kernel (bytes of LDS)
constexpr int ND_LDS_MAX = 65536;
__host__ __device__ inline int acc_rows(int R) { return R < ACC_LDS_R ? R : ACC_LDS_R; }

// order-preserving unsigned key of a double (larger value, larger key)
__host__ __device__ inline unsigned long long ordered_key(double x)
{
    unsigned long long b;
    __builtin_memcpy(&b, &x, 8);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double from_ordered_key(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    double x;
    __builtin_memcpy(&x, &b, 8);
    return x;
}

// Whether the main list keeps its sort keys. With one instance the sort key
// is the key's hash: for keys of up to two words it is recomputed where it is
// needed (cheaper than 8 bytes per entry moved twice per iteration); longer
// keys would turn each random probe of the merge partition into W scattered
// loads, so their sort keys stay stored. With several instances the sort key
// also holds the replica id and is always stored.
__host__ __device__ constexpr bool stored_skey(bool multi, int W) { return multi || W > 2; }

struct MainList {
    uint64_t *skey;  // sort key, kept when stored_skey(R > 1, W)
    uint64_t *key;   // word-major: key[w * cap + i]
    int32_t *pop;
    double *kdiag;   // H_ii - H_00
    int32_t *dslot;  // index in the deterministic space, -1 if not in it (kept while the space is active)
    int32_t *natt;   // spawning attempts for the next iteration
};

struct SpawnList {
    uint64_t *skey;   // sort key (replica | hash)
    uint64_t *rec;    // records of W + 1 words: key words, then amp | init << 32
    uint64_t *skey2;  // radix ping-pong
    uint32_t *idx;
    uint32_t *idx2;
};

struct UniqList {
    uint64_t *skey;
    uint64_t *key;  // word-major
    long long *sum;
    uint32_t *flag;
};

struct DetSpace {
    int32_t n;            // D (per replica equal; total = n * R)
    int32_t precision;
    int32_t npad;         // D rounded up to 32 (MFMA k steps)
    int32_t check_period; // split mode: FP64 check every check_period iterations
    int32_t shared;       // one D (and one K_DD) for all replicas
    int32_t nk;           // number of K_DD matrices: 1 if shared, else R
    const double *K;      // [nk][n][n] FP64 K_DD (replica-major)
    uint16_t *Khi;        // bf16 planes [nk][npad][npad], zero padded
    uint16_t *Klo;
    uint16_t *Chi;        // bf16 planes of the amplitudes [R][npad]
    uint16_t *Clo;
    double *yref;         // [R*n] FP64 projection of a checked iteration
    int32_t *pos;         // [R*n] position in the current main list
    const uint64_t *h64;  // [R*n] determinant hashes (for the rounding stream)
    double *c;            // [R*n] start-of-iteration populations
    double *y;            // [R*n] last projection
    long long *delta;     // [R*n] rounded projection increments
    const uint64_t *skey_sorted;  // [R*n] sorted (skey) for membership tests
    const uint64_t *key_sorted;   // [W][R*n]
};

// The part of a spawned-list segment that lies in one reduction tile when the
// segment's head is in an earlier tile (at most one per tile): added to the
// segment's total after the reduction.
struct BoundaryPart {
    long long sum;
    long long seg;
    uint32_t flag;
    uint32_t valid;
    long long pad;
};

struct Work {
    Ctl *ctl;
    EstAcc *acc;        // [R]
    EstAcc *hist;       // [HIST][R]
    double *shift;      // [R]
    const RepParams *rep;  // [R]
    const DevSys *sys;     // [n_sys]
    long long *att_off;    // [main_cap + 1]
    long long *span_lo;    // [spans + 1]
    long long *mpart;      // merge partition [tiles + 1]
    uint8_t *newdet;       // [main_cap]: 1 where the merge wrote a new determinant (K_jj still to compute)
    BoundaryPart *bpart;   // [reduction tiles]
    unsigned long long *st_scan, *st_sort, *st_red, *st_merge, *st_att;  // look-back status
    // per-block estimator partials of the reduction and the merge:
    // [block][acc_rows(R)][EST_FIELDS], folded into acc by the epilogue
    long long *part_red, *part_mrg;
    MainList cur, nxt;
    SpawnList sp;
    UniqList u;
    DetSpace ds;
    long long main_cap, spawn_cap, span_cap;
    int32_t R, rb, W, hist_len;
    uint64_t hmask;  // hash bits that enter a sort key (all but in collision tests)
    int32_t tau_search;  // track the maxima of the time-step search (per replica)
    int32_t lds_tables;  // bytes of UEG tables the spawn kernel stages in LDS (0: read from global)
    int32_t lds_diag;    // bytes of diagonal tables the new-determinant kernel stages in LDS
    // method: 0 FCIQMC; density matrices on pair keys (Sec. 2.3): 1 DMQMC
    // (both ends spawn, 2 attempts per walker unit), 2 IP-DMQMC (the ket end)
    int32_t dm;
    // CCMC (Sec. 2.2): truncation level of the excitors (0: not CCMC), the
    // exclusive prefix of |N_i| over the current list (reference masked),
    // its look-back status words and the queue of singles of the new list
    int32_t ccmc_trunc;
    int32_t single_cap;
    long long *ccmc_cum;        // [main_cap + 1]
    unsigned long long *st_ccmc;
    uint64_t *single_key;       // word-major [W][single_cap]
    int32_t *single_pop;        // [single_cap]
};

// launch geometry of the persistent kernels
struct Grids {
    int scan, part, spawn, hist, sort, reduce, fixup, merge, det;
    int spawn_lds;  // dynamic LDS bytes of the spawn kernel
    int newdiag;    // blocks of the new-determinant diagonal kernel
    // tile shapes (compile-time variants chosen at run time; results do not
    // depend on them): spawning attempts per thread (2, 4, 8; keys of up to two
    // words), merge positions per thread (1, 2, 4; keys of up to two words),
    // radix-sort keys per thread (8, 12, 16)
    int spawn_i = 4, merge_i = 2, sort_i = 12;
    int ccmc = 1024;  // blocks of the cluster-sampling kernel
};

// kernels of one iteration, in launch order (per-kernel timing slots; the
// two CCMC slots are empty for the other methods)
constexpr int N_KERNEL_SLOTS = 24;
// enqueue one whole iteration on a stream (ev: N_KERNEL_SLOTS + 1 events or nullptr)
hipError_t enqueue_iteration(const Work &w, int kind, const Grids &g, hipStream_t s, hipEvent_t *ev);
// CCMC stages: 0 = prefix of |N_i| and composite-cluster spawns (after the
// spawn kernel), 1 = singles-pair estimator of the new list (after the
// merge), 2 = the same for the current list (set-up)
hipError_t enqueue_ccmc(int stage, int kind, const Work &w, const Grids &g, hipStream_t s);
// set-up work: 0 = H_00 of every system, 1 = K_ii - H_00, attempt counts and
// attempt offsets of the current list of n entries, 2 = K_DD of the
// deterministic space
hipError_t enqueue_setup(int what, int kind, const Work &w, DevSys *sys, int n_sys, MainList L, long long n,
                         const uint64_t *dk, double *K, hipStream_t s);
// resident blocks per compute unit of a persistent kernel: 0 sort pass,
// 1 merge (keys of up to two words), 2 reduce, 3 attempt scan, 4 spawn,
// 5 merge (longer keys)
int occupancy_blocks(int which);

}  // namespace fq
