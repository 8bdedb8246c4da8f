/*
 * FCIQMC oracle: a plain, single-threaded CPU definition of one projector
 * iteration (spawning, death/cloning, annihilation with the initiator rule,
 * semi-stochastic projection, estimators, shift update), and of the same
 * iteration for the density-matrix and coupled cluster methods.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its binding) never calls it and shares no code with it.
 *
 * Paper: Spencer et al., "The HANDE-QMC project: open-source stochastic
 * quantum chemistry from the ground state up" (arXiv:1811.11679).
 *   propagation              Sec. 2.1, eq. (fciqmc), shift in the same section
 *   spawning / death /
 *   annihilation             Sec. 2.4 (commonality between the methods)
 *   initiator approximation  Sec. 2.1, last paragraph
 *   real (fixed-precision)
 *   weights                  Sec. 2.1 and the bibnote of Sec. 2.4
 *   semi-stochastic          Sec. 2.1; tutorial appendix, semi_stoch block
 *   projected energy         tutorial appendix, E_corr estimator
 *   sorted main list, hash   appendix "Parallelization"
 *   density matrix (DMQMC,
 *   IP-DMQMC)                Sec. 2.3, eqs. (dmqmc) and (ipdmqmc); Sec. 2.4
 *   coupled cluster (CCMC)   Sec. 2.2, eq. (ccmc); Sec. 2.4
 *
 * Parity pins (see the tests): brute-force second-quantised Hamiltonian,
 * exact diagonalisation, exhaustive generator enumeration, the rocRAND
 * Philox4x32-10 implementation, expectation values of the stochastic steps,
 * Jordan-Wigner excitor products and deterministic coupled cluster energies.
 */
#ifndef FQ_ORACLE_H
#define FQ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXW 8

enum { OR_HUBBARD = 1, OR_UEG = 2, OR_MOLECULAR = 3 };
enum { OR_EXGEN_HUB = 1, OR_EXGEN_UEG = 2, OR_EXGEN_HEATBATH = 3 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_EOVERFLOW = -3, OR_ENOREF = -7 };

typedef struct or_sys or_sys;
typedef struct or_run or_run;

typedef struct {
    double tau;
    uint64_t seed;
    int32_t replica_id;
    double init_pop;            /* walkers on D_0 at start */
    double target_population;   /* walkers */
    int32_t shift_period;       /* A (mc_cycles) */
    double shift_damping;       /* zeta */
    double initial_shift;       /* S_0, relative to H_00 */
    int32_t excit_gen;
    double p_single;
    int32_t initiator;
    double initiator_threshold; /* n_add, walkers */
    int32_t fixed_point_bits;   /* 0: integer walkers, b: resolution 2^-b */
    double spawn_cutoff;        /* walkers, real mode only */
    int32_t ss_size;            /* 0: no semi-stochastic */
    int32_t ss_start_iteration;
    int32_t ss_shared;          /* 1: D chosen jointly with other runs (or_runs_select_shared) */
    int32_t tau_search;         /* 1: lower tau on the fly (see step_once) */
    int32_t method;             /* OR_FCIQMC, OR_DMQMC, OR_IPDMQMC or OR_CCMC */
    int32_t ccmc_truncation;    /* CCMC: highest excitation level of an excitor (2: CCSD, ...) */
} or_qmc;

/* Methods (Sec. 2.1 FCIQMC; Sec. 2.2 CCMC; Sec. 2.3 DMQMC and
 * interaction-picture DMQMC). The density-matrix methods sample pairs
 * (D_i, D_j): a key of 2W words, the bra's W words first, then the ket's.
 * CCMC samples excitor amplitudes on the determinants D_i = a_i D_0 up to the
 * truncation level (the reference's entry holds t_HF = N_0). */
enum { OR_FCIQMC = 0, OR_DMQMC = 1, OR_IPDMQMC = 2, OR_CCMC = 3 };

/* estimators of the last completed iteration */
typedef struct {
    int64_t iteration, n_walkers_units, n_occupied, n_spawned, ref_pop_units;
    int64_t n_sign_flips, n_rejected_units, n_spawn_events;
    int64_t death_sum, spawn_sum, rejected_sum; /* signed unit totals of the last iteration */
    int32_t vary_shift, status;
    double shift, proj_numerator, proj_energy, e_ref;
    int64_t num_limbs[4];
    /* CCMC: sum over pairs of singles a < b of H_0,ab sgn(a_a a_b D_0) N_a N_b
       (units 2^-2b, exact limbs at 2^-64); proj_energy adds it over N_0^2 */
    int64_t pair_limbs[4];
    double tau;             /* time step in force for the next iteration */
    double spawn_ratio_max; /* largest |H_ji| / p_gen of any attempt so far (tau search only) */
    int64_t n_cluster_spawns; /* CCMC: spawn records of the sampled composite clusters, last iteration */
} or_estimators;

/* Philox4x32-10, Salmon et al. (SC'11) */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* MurmurHash64A over the 8W bytes of a bit string (little-endian words) */
uint64_t or_hash64(const uint64_t *w, int W);

or_sys *or_hubbard_new(int n_sites, int periodic, double t, double U, int n_alpha, int n_beta);
or_sys *or_ueg_new(double rs, int ecut_n2, int n_alpha, int n_beta);
or_sys *or_molecular_new(int n_orb, const double *h1, const double *eri, int n_alpha, int n_beta);
void or_sys_free(or_sys *s);
/* iout: kind, n_spatial, n_so, W, nel, n_alpha, n_beta; dout: H00, L, k2, vc */
void or_sys_info(const or_sys *s, int32_t *iout, double *dout);
void or_sys_reference(const or_sys *s, uint64_t *key);
void or_ueg_orbitals(const or_sys *s, int32_t *nvec);
int64_t or_heatbath_size(const or_sys *s);
double or_hij(const or_sys *s, const uint64_t *bra, const uint64_t *ket);
double or_diag(const or_sys *s, const uint64_t *key);

/* One excitation draw with explicit random words: w[0..3] is the tag-0 block,
 * w[4..7] the tag-1 block. Returns 1 and fills child/pgen/hij, or 0 (null). */
int or_exgen(const or_sys *s, int exgen, double p_single, const uint64_t *key,
             const uint32_t *w, uint64_t *child, double *pgen, double *hij);

or_run *or_run_new(const or_sys *s, const or_qmc *q);
void or_run_free(or_run *r);
int or_run_step(or_run *r, int n_iter);
/* one deterministic space for several runs of one system (qmc.ss_shared = 1):
   the ss_size determinants of largest sum over the runs of |n| (key ascending
   on ties), inserted with n = 0 where a run does not hold them */
int or_runs_select_shared(or_run **runs, int n_runs);
void or_run_estimators(const or_run *r, or_estimators *out);
int64_t or_run_size(const or_run *r);
void or_run_export(const or_run *r, uint64_t *keys, int32_t *pops);
int or_run_import(or_run *r, const uint64_t *keys, const int32_t *pops, int64_t n,
                  double shift, int64_t iteration, int32_t vary, int64_t n_prev);
int64_t or_run_n_spawns(const or_run *r);
void or_run_spawns(const or_run *r, uint64_t *keys, int32_t *amps, uint8_t *init);
int64_t or_run_detspace(const or_run *r, uint64_t *keys);
/* last deterministic projection y = K_DD n_D (FP64, fixed order), D order */
void or_run_last_projection(const or_run *r, double *y);
/* CCMC: a_{e_1} ... a_{e_n} D_0 = sign D for the excitors of the n keys ex
   (n x W words; a_e D_0 = +D_e); returns sign (+1/-1) and fills out, or 0
   when the product vanishes */
int or_cluster_collapse(const or_sys *s, const uint64_t *ex, int n, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
