"""Run parameters of the synthetic workloads (plain values, no arithmetic).

Each entry gives the system description and the qmc parameters in the units of
the paper's input tables (tutorial appendix): walkers, Hartree, iterations.
"""

# 1D Hubbard ring, 8 sites, U/t = 4, half filling: 4900 determinants
HUBBARD8 = dict(
    system=dict(kind="hubbard", n_sites=8, periodic=1, t=1.0, U=4.0, n_alpha=4, n_beta=4),
    qmc=dict(tau=0.01, rng_seed=7, init_pop=500.0, target_population=1e4, shift_period=10,
             shift_damping=0.05, initial_shift=-4.0, initiator=0, fixed_point_bits=0, spawn_cutoff=0.0),
    iterations=2000,
)

# 3D uniform electron gas: 14 electrons, rs = 1, 57 plane waves (114 spin-orbitals)
UEG14 = dict(
    system=dict(kind="ueg", rs=1.0, ecut_n2=5, n_alpha=7, n_beta=7),
    qmc=dict(tau=0.002, rng_seed=7, init_pop=5e5, target_population=1e7, shift_period=10,
             shift_damping=0.05, initial_shift=0.0, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1),
    iterations=5000,
    # the benchmark times the last 1000 of the 5000 iterations: the population
    # reaches the target near iteration 150 and the shift has settled by 1500
    equilibration=4000,
)

# molecular-like Hamiltonian: 30 orbitals, 8 + 8 electrons, heat-bath generator
MOL30 = dict(
    system=dict(kind="molecular", n_orb=30, n_alpha=8, n_beta=8),
    qmc=dict(tau=0.001, rng_seed=7, init_pop=5e5, target_population=1e7, shift_period=10,
             shift_damping=0.05, initial_shift=0.0, p_single=0.1, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1),
    semistoch=dict(size=2000, start_iteration=1000),
    iterations=2000,
)

# large UEG: 54 electrons, 251 plane waves (502 spin-orbitals). The target
# population holds the list at about 1.8e8 determinants; with the tutorial's
# damping 0.05 the initial growth (~7.5% per iteration) overruns any list of a
# few 1e8 entries before the shift responds, so the damping is 1.0.
UEG54 = dict(
    system=dict(kind="ueg", rs=1.0, ecut_n2=14, n_alpha=27, n_beta=27),
    qmc=dict(tau=0.0005, rng_seed=7, init_pop=1e4, target_population=2e7, shift_period=10,
             shift_damping=1.0, initial_shift=0.0, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1),
    semistoch=dict(size=8192, start_iteration=900),
    iterations=500,
    # untimed warm-up before the 500 timed iterations; the list is at its
    # working size (about 1.8e8 determinants) from iteration ~300 on
    equilibration=1000,
)

# coupled cluster Monte Carlo at CCSD on the 14-electron gas (the paper's UEG
# CCMC comparison, Sec. 4.3): about 1.8e3 amplitudes, N_ex / N_0 near 9 at
# the CCSD amplitudes, so 1e6 walkers on D_0 hold about 1e7 in total; the
# population settles within a few hundred iterations
UEG14_CCSD = dict(
    system=dict(kind="ueg", rs=1.0, ecut_n2=5, n_alpha=7, n_beta=7),
    qmc=dict(tau=0.002, rng_seed=7, init_pop=1e6, target_population=8e6, shift_period=10,
             shift_damping=0.05, initial_shift=0.0, initiator=0, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1, method=3, ccmc_truncation=2),
    equilibration=1000,
)

UEG_ECUT_FOR_BASIS = {19: 2, 27: 3, 57: 5, 123: 9}


def batch64(n_replicas=64, seed=7):
    """64 independent electron-gas instances of 14 electrons (7 + 7): rs and
    the basis size drawn uniformly from {0.5, 1, 2, 4} x {19, 27, 57, 123}
    plane waves, targets log-uniform in [1e5, 2e6] walkers, initial population
    target / 20, dtau = 0.002 min(1, rs^2) (energies grow as 1 / rs^2), one
    Philox stream per replica (key word 1 xor replica id); everything else as
    UEG14. Returns a list of (system, qmc) dicts."""
    from .synth import batched_ueg_draws
    out = []
    for r, (rs, m, tgt) in enumerate(batched_ueg_draws(n_replicas, seed)):
        system = dict(kind="ueg", rs=rs, ecut_n2=UEG_ECUT_FOR_BASIS[m], n_alpha=7, n_beta=7)
        qmc = dict(UEG14["qmc"], tau=0.002 * min(1.0, rs * rs), init_pop=tgt / 20.0, target_population=tgt,
                   replica_id=r)
        out.append((system, qmc))
    return out
