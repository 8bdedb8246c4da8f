/*
 * fciqmc.h -- C ABI of the MI355X FCIQMC hot path (one GPU, HIP, gfx950).
 *
 * One projector iteration of full configuration interaction quantum Monte
 * Carlo over a list of occupied Slater determinants held as bit strings with
 * signed fixed-point walker populations (Spencer et al., "The HANDE-QMC
 * project", arXiv:1811.11679):
 *   c_i(tau + dtau) = c_i(tau) - dtau sum_j <D_i|H - S|D_j> c_j(tau)
 * (Sec. 2.1, eq. fciqmc, with the shift S as a diagonal energy offset),
 * sampled by spawning, death/cloning and annihilation (Sec. 2.4), with real
 * fixed-precision weights (Sec. 2.1 and the weights bibnote), the initiator
 * approximation (Sec. 2.1), semi-stochastic propagation in a deterministic
 * space (Sec. 2.1; tutorial appendix, semi_stoch block), the projected-energy
 * estimator (tutorial appendix) and the sorted main list / spawned list of the
 * appendix "Parallelization".
 *
 * Conventions shared by every call:
 *  - Every function returns fq_status: 0 on success, a negative code on error.
 *    fq_last_error() returns a text for the last error of a context.
 *  - Host pointers (integral arrays, walker keys and populations) belong to
 *    the caller and are only read (or written, for export) during the call.
 *  - The device workspace belongs to the caller, must hold at least
 *    fq_workspace_bytes() bytes, be 256-byte aligned and outlive the context.
 *  - The HIP stream belongs to the caller; every device operation of a context
 *    is enqueued on it. Calls on one context must not run concurrently.
 *  - Bit strings: spin-orbital P = 2p + sigma (sigma 0 = alpha, 1 = beta) is bit
 *    P % 64 of 64-bit word P / 64; word 0 is least significant; a key holds W
 *    = ceil(n_spin_orbitals / 64) words, W in {1, 2, 4, 8} (3 is padded to 4,
 *    5..7 to 8). Keys are compared as unsigned big integers.
 *  - Populations are int32 multiples of 2^-b walkers (b = fixed_point_bits;
 *    b = 0 gives integer walkers).
 *
 * Errors: FQ_EINVAL (bad arguments; nothing is changed), FQ_ECAPACITY (a list
 * would exceed its capacity), FQ_EOVERFLOW (a population or spawn would exceed
 * int32), FQ_EHIP (a HIP runtime call failed), FQ_ESTATE (call out of order).
 * After FQ_ECAPACITY or FQ_EOVERFLOW from fq_step the walker lists are those
 * at the start of the failing iteration and the context can be exported.
 */
#ifndef FCIQMC_H
#define FCIQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fq_status;
#define FQ_OK 0
#define FQ_EINVAL (-1)
#define FQ_ECAPACITY (-2)
#define FQ_EOVERFLOW (-3)
#define FQ_EHIP (-4)
#define FQ_ESTATE (-5)
#define FQ_ENOREF (-6) /* CCMC: the reference determinant holds no walkers */

/* model systems (paper Sec. 4.3: uniform electron gas, Hubbard) and molecular
 * integrals (Sec. 3.1 and the tutorial appendix: h_pq and (pq|rs)) */
#define FQ_HUBBARD_REAL 1
#define FQ_UEG 2
#define FQ_MOLECULAR 3

/* excitation generators (Sec. 2.4 "system dependent"; heat bath, Sec. 2.1) */
#define FQ_EXGEN_HUB_UNIFORM 1
#define FQ_EXGEN_UEG_UNIFORM 2
#define FQ_EXGEN_HEATBATH_UNIFORM_SINGLES 3

#define FQ_SS_FP64 0       /* deterministic projection in FP64, fixed order */
#define FQ_SS_SPLIT_BF16 1 /* BF16 x3 split products, FP32 accumulation (MFMA) */

/* A system. Hubbard: 1D chain of n_sites, periodic or open, hopping t,
 * on-site U, real-space basis. UEG: plane waves n in Z^3 with |n|^2 <= ecut_n2
 * in a cubic box of side L = rs (4 pi N / 3)^(1/3), Coulomb 4 pi / (L^3 k^2),
 * k = 0 term excluded. Molecular: n_orb spatial orbitals, h1[p*n+q] and
 * eri[((p*n+q)*n+r)*n+s] = (pq|rs) in chemists' notation, both real and
 * symmetric, copied during fq_init_system. */
typedef struct {
    int32_t kind;
    int32_t n_alpha, n_beta;
    int32_t n_sites, periodic;
    double t, U;
    double rs;
    int32_t ecut_n2;
    int32_t n_orb;
    const double *h1;
    const double *eri;
} fq_system;

/* Run parameters, as the paper's qmc table (tutorial appendix). */
typedef struct {
    double tau;                 /* time step dtau */
    uint64_t rng_seed;          /* Philox key = (seed_lo, seed_hi ^ replica_id) */
    int32_t replica_id;
    double init_pop;            /* walkers placed on the reference at start */
    double target_population;   /* walkers; the shift varies once it is reached */
    int32_t shift_period;       /* A: iterations between shift updates (mc_cycles) */
    double shift_damping;       /* zeta */
    double initial_shift;       /* S at start, relative to H_00 */
    int32_t excit_gen;          /* FQ_EXGEN_* matching the system */
    double p_single;            /* heat-bath generator: probability of a single */
    int32_t initiator;          /* 1: initiator approximation on */
    double initiator_threshold; /* n_add, walkers (strict >) */
    int32_t fixed_point_bits;   /* b; 0 = integer walkers, else 3..20 (FQ_EINVAL otherwise:
                                   with b = 1, 2 an int32 population could need 2^28 or more
                                   spawning attempts, the limit of the random-number counter) */
    double spawn_cutoff;        /* walkers; real mode only */
    int32_t tau_search;         /* 1: the tutorial's tau_search, per instance. After each
                                   shift update of the instance its tau only decreases, to
                                   min(tau, 1 / max |H_ji| / p_gen over every attempt of the
                                   instance so far, 1 / (max K_ii - S) over the instance's
                                   entries of the last death step), each bound applying when
                                   positive. Export/import keep tau and the running maximum. */
    int32_t method;             /* FQ_FCIQMC, FQ_DMQMC, FQ_IPDMQMC or FQ_CCMC (the same for
                                   every instance of a context) */
    int32_t ccmc_truncation;    /* FQ_CCMC: highest excitation level of an excitor, 1..6
                                   (1: CCS, 2: CCSD, ...); ignored otherwise */
} fq_qmc;

/* Methods (Sec. 2.1; Sec. 2.3, eqs. dmqmc and ipdmqmc; Sec. 2.4). The
 * density-matrix methods sample pairs (D_i, D_j) holding rho_ij: a key of two
 * words, the bra's determinant (word 0) and the ket's (word 1), so the system
 * must have at most 64 spin-orbitals. Annihilation is the FCIQMC one on these
 * keys. DMQMC (symmetrised Bloch equation): each pair makes ceil(|n| 2^-b)
 * spawning attempts at each end (attempt 2k acts on the bra, 2k + 1 on the
 * ket) with amplitude (tau / 2)|H| / p_gen per walker, and dies with
 * (K_ii + K_jj) / 2 - S. IP-DMQMC (H^0 the diagonal part of H, df/dtau =
 * H^0 f - f H): only the ket end spawns (amplitude tau |H| / p_gen), death
 * with K_jj - K_ii - S. The initial list is round(init_pop 2^b) units on
 * (D_0, D_0); a beta loop starts from the caller's sample of the identity (or
 * of e^{-beta H^0}) given to fq_import_walkers. Estimators: ref_pop_units is
 * the trace sum_i rho_ii and proj_numerator / num_limbs Tr(rho H) =
 * sum rho_ij H_ji (H_ii on the diagonal, absolute), so proj_energy is the
 * thermal energy Tr(rho H) / Tr(rho). Not with the initiator rule, a
 * deterministic space or tau_search (FQ_EINVAL). */
#define FQ_FCIQMC 0
#define FQ_DMQMC 1
#define FQ_IPDMQMC 2

/* Coupled cluster Monte Carlo (Sec. 2.2, eq. ccmc; Sec. 2.4). The list holds
 * excitor amplitudes N_i on D_i = a_i D_0 up to the truncation level
 * (a_i D_0 = +D_i) and t_HF = N_0 on D_0; Psi = N_0 exp(T / N_0) D_0 with
 * T = sum_i N_i a_i. Each iteration: every entry spawns and dies as an
 * FCIQMC parent (spawns beyond the truncation level are not made); then
 * n_c = ceil(N_ex 2^-b) composite clusters are sampled, N_ex = sum |N_i|
 * over the excitors: size s in [2, truncation + 2] with p(s) = 2^-(s-1) (the
 * largest size taking the remainder), s excitors with probability
 * |N_i| / N_ex each in list order (64-bit hash, then key), the product
 * a_{e_1}...a_{e_s} D_0 = sgn D (zero when two excitors share a hole or a
 * particle); the term of weight sgn N_0 (N_ex / |N_0|)^s / (p(s) s! n_c)
 * makes one spawning attempt from D and, when D is within the truncation
 * level, adds its death step -dtau (K_DD - S) w as a spawn onto D. Spawns
 * and annihilation are FCIQMC's. Random numbers of cluster c: Philox under
 * (seed_lo, seed_hi ^ replica_id ^ 2^31), counter (tag, draw, t, c). The
 * projected energy is sum_j H_0j t~_j / N_0 where t~_j = <D_j|Psi> holds, for
 * a double, the products (1 / N_0) sgn N_a N_b of pairs of singles
 * (fq_estimators_t.pair_limbs). One instance per context; not with the
 * initiator rule, a deterministic space or tau_search (FQ_EINVAL). A
 * step whose reference holds no walkers fails with FQ_ENOREF; fq_step refuses
 * to start a block of iterations with 2^36 or more units of walkers
 * (FQ_EOVERFLOW: the prefix of |N_i| is carried in 38-bit words). */
#define FQ_CCMC 3

/* Semi-stochastic block (tutorial appendix, semi_stoch = {size,
 * start_iteration, space = "high"}): the size most highly weighted
 * determinants at the end of iteration start_iteration form D. */
typedef struct {
    int32_t size;
    int32_t start_iteration;
    int32_t precision;    /* FQ_SS_FP64 or FQ_SS_SPLIT_BF16 */
    int32_t check_period; /* split mode: every check_period iterations the FP64
                             projection is also computed and the largest error
                             of the split result, relative to sum_j |K_ij||c_j|,
                             is reported in fq_estimators_t.ss_error (0: never) */
    int32_t shared;       /* 0: each instance selects its own D. 1: one D for all
                             instances (all must describe the same system): the
                             size determinants of largest summed |n| over the
                             instances (key ascending on ties), present in every
                             instance's list (with n = 0 where unoccupied), so that
                             K_DD C over all instances is one matrix product */
} fq_semistoch;

/* Estimators of one iteration of one instance (tutorial appendix: shift,
 * number of walkers, projected-energy numerator sum_j H_0j N_j and
 * denominator N_0). Walker quantities are in units of 2^-b walkers except
 * proj_numerator, which is in walkers. */
typedef struct {
    int64_t iteration;
    int64_t n_walkers_units;  /* sum |n_i| */
    int64_t n_occupied;       /* determinants in the main list */
    int64_t n_spawned;        /* spawn events this iteration */
    int64_t ref_pop_units;    /* n_0 */
    int64_t n_sign_flips;     /* death steps that changed a population's sign */
    int64_t n_rejected_units; /* sum |A| of segments refused by the initiator rule */
    int64_t n_spawn_events;   /* distinct spawned determinants */
    int64_t death_sum, spawn_sum, rejected_sum; /* signed unit totals */
    int32_t vary_shift, status;
    double shift;             /* relative to H_00 */
    double proj_numerator;    /* walkers x Hartree */
    double proj_energy;       /* numerator / N_0 (correlation energy); NaN if N_0 = 0 */
    double e_ref;             /* H_00 */
    int64_t num_limbs[4];     /* exact fixed-point numerator (2^-64 resolution), units */
    double ss_error;          /* split projection: max_i |y_i - y_i(FP64)| / sum_j |K_ij||c_j|
                                 of the last checked iteration (0 if none) */
    double ss_error_bound;    /* a priori bound of that ratio for the BF16 x3 / FP32 scheme */
    double tau;               /* time step of the next iteration (tau_search may lower it) */
    double spawn_ratio_max;   /* tau_search: largest |H_ji| / p_gen of any attempt so far, as of
                                 the end of the fq_step call (0 without tau_search) */
    int64_t pair_limbs[4];    /* CCMC: exact fixed-point (2^-64) sum over pairs of singles a < b
                                 of H_0,ab sgn(a_a a_b D_0) N_a N_b (units^2); proj_numerator and
                                 proj_energy add it divided by N_0. Zero otherwise. */
    int64_t n_cluster_spawns; /* CCMC: spawn records written by the sampled composite clusters
                                 this iteration (their spawns and death steps); part of n_spawned */
} fq_estimators_t;

typedef struct fq_ctx fq_ctx;

/* Bytes of device workspace needed for n_instances replicas that share one
 * system shape (same kind and key width), with main_capacity determinants and
 * spawn_capacity spawned walkers summed over the instances. qmc (may be NULL,
 * meaning FCIQMC) gives the method, which sets the key width. */
size_t fq_workspace_bytes(const fq_system *sys, const fq_qmc *qmc, const fq_semistoch *ss,
                          int32_t n_instances, int64_t main_capacity, int64_t spawn_capacity);

/* Creates a context for n_instances independent replicas (arrays sys[], qmc[]
 * and, if not NULL, ss[] of that length) that advance together. Each replica
 * starts with round(init_pop 2^b) units on its reference determinant (Hubbard:
 * alpha on sites 0,2,4,..., beta on 1,3,5,...; UEG and molecular: aufbau). */
fq_status fq_init_system(fq_ctx **out, const fq_system *sys, const fq_qmc *qmc,
                         const fq_semistoch *ss, int32_t n_instances, int64_t main_capacity,
                         int64_t spawn_capacity, void *d_workspace, size_t ws_bytes,
                         void *hip_stream);

/* Allocation-free variant of fq_init_system, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The context's workspace is a static device
 * array of FQ_STATIC_WORKSPACE_BYTES that the library holds on every device it
 * runs on until the process ends; the call makes no hipMalloc, hipHostMalloc,
 * hipFree or other allocating HIP or torch call (its host staging buffers are
 * plain host memory). Arguments and results are those of fq_init_system
 * without d_workspace / ws_bytes; the array of the current device is used.
 * Errors: FQ_ECAPACITY (nothing created) when fq_workspace_bytes() of the
 * arguments exceeds FQ_STATIC_WORKSPACE_BYTES (a few 1e4 determinants: the
 * 8-site Hubbard ring with 16384 determinants and 65536 spawns needs 7.3 MiB);
 * FQ_ESTATE when a context made by this call on the same device has not yet
 * been destroyed (every such context would share the one array, and calls on
 * two of them would race, so only one may live per device); FQ_EINVAL as for
 * fq_init_system. The array keeps the contents of the last context; every part
 * that must start at zero is cleared by this call. fq_destroy gives the array
 * back. */
#define FQ_STATIC_WORKSPACE_BYTES (16u << 20)
fq_status fq_init_system_static(fq_ctx **out, const fq_system *sys, const fq_qmc *qmc,
                                const fq_semistoch *ss, int32_t n_instances, int64_t main_capacity,
                                int64_t spawn_capacity, void *hip_stream);

/* Advances every replica by n_iterations projector iterations (spawning,
 * death/cloning, semi-stochastic projection, annihilation with the initiator
 * rule, estimators, and the shift update every shift_period iterations:
 * S <- S - zeta / (A dtau) ln(N_w(t) / N_w(t - A)) once N_w reached target).
 * Returns after the work is enqueued and the host-side shift logic has run;
 * estimators of every iteration are available afterwards. */
fq_status fq_step(fq_ctx *ctx, int32_t n_iterations);

/* Estimators of the last completed iteration of one instance. */
fq_status fq_estimators(const fq_ctx *ctx, int32_t instance, fq_estimators_t *out);

/* Estimators of the last n iterations (up to the last fq_step call), oldest
 * first; *n_out receives the number written. */
fq_status fq_estimator_history(const fq_ctx *ctx, int32_t instance, fq_estimators_t *out,
                               int32_t cap, int32_t *n_out);

/* Copies the main list of one instance to host arrays, sorted by key:
 * keys[i*W + w], pops[i]. cap is the capacity in determinants. */
fq_status fq_export_walkers(const fq_ctx *ctx, int32_t instance, uint64_t *keys, int32_t *pops,
                            int64_t cap, int64_t *n_out);

/* Replaces the main list of one instance (distinct keys, any order; zero
 * populations are dropped) and sets its shift state and iteration counter
 * (all instances share the counter: the same value must be given for each).
 * If the semi-stochastic block is active and iteration >= start_iteration,
 * the deterministic space is chosen from the imported list. */
fq_status fq_import_walkers(fq_ctx *ctx, int32_t instance, const uint64_t *keys,
                            const int32_t *pops, int64_t n, double shift, int64_t iteration,
                            int32_t vary_shift, int64_t n_prev);

/* Shift state of one instance after the last completed iteration: the shift
 * S (Hartree, relative to H_00), the population (units) at the last shift
 * update and whether S is being varied. With fq_export_walkers and
 * fq_estimators this is everything fq_import_walkers needs to continue the run
 * exactly (Sec. 2.1 and the tutorial appendix: S is updated every A iterations from the ratio of
 * populations). Any output pointer may be NULL. */
fq_status fq_shift_state(const fq_ctx *ctx, int32_t instance, double *shift, int64_t *n_prev,
                         int32_t *vary_shift);

/* Spawned walkers of the last iteration of one instance (unordered):
 * keys[i*W + w], amps[i] (units), init[i] (1 if the parent was an initiator). */
fq_status fq_export_spawns(const fq_ctx *ctx, int32_t instance, uint64_t *keys, int32_t *amps,
                           uint8_t *init, int64_t cap, int64_t *n_out);

/* Deterministic space of one instance in D order (|n| descending, key
 * ascending at selection) and the last projection y = K_DD n (FP64 or
 * split precision); either pointer may be NULL. */
fq_status fq_detspace(const fq_ctx *ctx, int32_t instance, uint64_t *keys, double *last_y,
                      int64_t cap, int64_t *n_out);

/* Key width W and (kind, n_spin_orbitals, H_00) of a context. */
fq_status fq_info(const fq_ctx *ctx, int32_t *W, int32_t *n_spin_orbitals, double *e_ref);

/* Per-stage device time of the last fq_step call, in milliseconds, summed
 * over its iterations, measured with HIP events on the context's stream:
 * [0] attempt partition, [1] spawning, [2] radix sort, [3] segmented reduction,
 * [4] merge with death and estimators, [5] deterministic projection,
 * [6] whole iterations. Timing is recorded only after fq_set_timing(ctx, 1). */
fq_status fq_set_timing(fq_ctx *ctx, int32_t on);
fq_status fq_stage_times(const fq_ctx *ctx, double *ms7);

/* Per-kernel device time of the last fq_step call (timing on), summed over its
 * iterations, one slot per launch of an iteration in launch order: begin,
 * attempt partition, spawn, sort histogram, sort passes 0..7,
 * reduce, collision fix-up, reduce (repeat), projection gather, projection,
 * projection check, merge partition, merge, new-determinant diagonals, end.
 * *n_slots receives the slot count (22) and
 * *n_iterations the number of timed iterations. */
fq_status fq_kernel_times(const fq_ctx *ctx, double *ms, int32_t cap, int32_t *n_slots,
                          int64_t *n_iterations);

/* Device time of each iteration of the last fq_step call made with timing on
 * (first event of the iteration to its last), ms, oldest first; *n_out
 * receives the number written (at most cap). */
fq_status fq_iteration_times(const fq_ctx *ctx, double *ms, int64_t cap, int64_t *n_out);

/* Graph replay: with on = 1, every block of shift_period iterations between
 * two host shift updates is captured once into a HIP graph (per main-list
 * parity) and replayed with one launch. The stream given to fq_init_system
 * must not be the legacy default stream. Timing (fq_set_timing) launches
 * kernels one by one and takes precedence. */
fq_status fq_set_graph(fq_ctx *ctx, int32_t on);

/* Sort-key truncation, for tests of the hash-collision path (the annihilation
 * of Sec. 2.4 must combine walkers on one determinant however the list is
 * ordered). Only the top `bits` (1..64) bits of each determinant's 64-bit hash
 * then enter its sort key, so that many determinants share a sort key and
 * ties are broken by the determinant itself, in the main list and in the
 * spawned list (collision fix-up and repeated reduction every iteration).
 * Results are unchanged: the random streams are keyed by the full hash.
 * Needs two or more instances (FQ_EINVAL otherwise: a single instance's
 * kernels use the sort key as the hash) and must precede the deterministic
 * space (FQ_ESTATE). The current list is re-sorted on the host. A run of
 * equal sort keys holding more than 64 determinants fails the iteration
 * with FQ_ESTATE. */
fq_status fq_set_sort_key_bits(fq_ctx *ctx, int32_t bits);

/* Launch geometry of the persistent kernels, in blocks: [0] spawn, [1] merge,
 * [2] radix-sort pass, [3] segmented reduction, [4] new-determinant
 * diagonals. A value <= 0 keeps the current one. Results do not depend on
 * the geometry (work is taken by ticket or grid stride); only speed does. */
fq_status fq_set_launch(fq_ctx *ctx, const int32_t *blocks, int32_t n);
fq_status fq_get_launch(const fq_ctx *ctx, int32_t *blocks, int32_t n);

/* Tile shapes of the persistent kernels, among variants compiled into the
 * library: [0] spawning attempts per thread (2, 4 or 8; tiles of 256 threads),
 * [1] merge positions per thread (1, 2 or 4; tiles of 512 threads), [2]
 * radix-sort keys per thread (8, 12 or 16; tiles of 256 threads). [0] and [1]
 * apply to determinant keys of one or two words (longer keys and pair keys
 * use 2 and 2, resp. 4 and 2); [2] to every context. Defaults 4, 2, 12. A value
 * <= 0 keeps the current one; any other value outside the list is FQ_EINVAL
 * (nothing changes). Results do not depend on the shapes (tiles only
 * partition the work; every prefix crossing tiles is exact); only speed does.
 * Changing them drops the captured graphs. */
fq_status fq_set_tiles(fq_ctx *ctx, const int32_t *tiles, int32_t n);
fq_status fq_get_tiles(const fq_ctx *ctx, int32_t *tiles, int32_t n);

/* On-the-fly blocking analysis (Sec. 3.1: the reblocking of Flyvbjerg and
 * Petersen, accumulated as the data arrive, so that a run can stop once a
 * requested statistical error is reached). Host-only: no device call, no
 * context needed. An accumulator holds n_series (1..64) series observed
 * together and n_levels (1..62) blocking levels: level k holds the means of
 * consecutive blocks of 2^k observations (pairwise averages of level k - 1;
 * an incomplete last block is left out, as in the post-hoc analysis). Memory
 * is O(n_levels * n_series^2), independent of the number of observations.
 *
 * fq_reblock_create: *out receives the accumulator (owned by the caller,
 *   released by fq_reblock_destroy); FQ_EINVAL for sizes out of range.
 * fq_reblock_add: x[n_series], one observation of every series; FQ_EINVAL for
 *   a non-finite value (nothing is recorded).
 * fq_reblock_level: *n_blocks receives the number of complete blocks at the
 *   level; mean[n_series] (optional) their means; cov[n_series * n_series]
 *   (optional, row-major) the sample covariance of the block values (divided
 *   by n_blocks - 1; NaN below two blocks). The variance of the mean of
 *   series s at that level is cov[s * n_series + s] / n_blocks.
 * fq_reblock_optimal: *level receives the smallest level whose block length
 *   B = 2^k satisfies B^3 > 2 n (e_k / e_0)^4 (n observations, e_k the
 *   standard error of the mean from level k; Lee, Needs and Towler's
 *   criterion), or -1 when no level satisfies it yet (not enough data).
 * fq_reblock_ratio: mean(num) / mean(den) at a level and its first-order
 *   standard error from the block covariances (the projected energy:
 *   numerator and reference population averaged separately, then divided);
 *   *err is NaN below two blocks or for a zero denominator. */
typedef struct fq_reblock fq_reblock;
fq_status fq_reblock_create(fq_reblock **out, int32_t n_series, int32_t n_levels);
fq_status fq_reblock_add(fq_reblock *rb, const double *x);
fq_status fq_reblock_level(const fq_reblock *rb, int32_t level, int64_t *n_blocks, double *mean, double *cov);
fq_status fq_reblock_optimal(const fq_reblock *rb, int32_t series, int32_t *level);
fq_status fq_reblock_ratio(const fq_reblock *rb, int32_t level, int32_t num, int32_t den, double *ratio,
                           double *err);
void fq_reblock_destroy(fq_reblock *rb);

const char *fq_last_error(const fq_ctx *ctx);
void fq_destroy(fq_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
