"""Semi-stochastic energies: split precision against FP64 at the molecular
workload's size.

The 30-orbital molecular-like system (8 + 8 electrons, heat-bath doubles,
1/256 weights, initiator 3, target 1e7 walkers) with a deterministic space of
the 2000 most highly weighted determinants (paper Sec. 2.1, semi-stochastic
propagation; tutorial appendix, semi_stoch). One FP64 run is equilibrated for
3000 iterations and its list exported when the space is chosen; a
split-precision run (BF16 x3 products, FP32 accumulation on MFMA) imports that
state with the same random keys. Both then run 3000 iterations. The split projection changes the walker
dynamics only through rounding differences of about 1e-5 relative, so the two
reblocked projected energies must agree within two combined standard errors.
"""
import math

import numpy as np
import pytest

from gpu_helpers import say
from oracle import reblock
from paper_1811_11679_amd import synth, workloads

pytestmark = pytest.mark.gpu

T0, N_ITER, D = 3000, 3000, 2000


def _energy(hist):
    """Reblocked ratio of the averaged numerator and reference population: at
    the criterion's level for both series, or, if a series has not reached it,
    at the level of at least 16 blocks with the largest error (the blocking
    error grows with the level until the blocks decorrelate)."""
    x = np.array([[h["proj_numerator"], h["ref_pop_units"] / 256.0] for h in hist])
    lv = reblock.block_levels(x)
    ks = [reblock.optimal_level(lv, 0), reblock.optimal_level(lv, 1)]
    if min(ks) >= 0:
        k = max(ks)
    else:
        cand = [j for j in range(len(lv)) if lv[j][0] >= 16]
        k = max(cand, key=lambda j: reblock.ratio(lv, j, 0, 1)[1])
    e, err = reblock.ratio(lv, k, 0, 1)
    return e, err, k


def test_split_energy_within_two_sigma_of_fp64_at_d2000():
    from paper_1811_11679_amd import fciqmc as F
    h1, eri = synth.molecular_integrals()
    w = workloads.MOL30
    q = dict(w["qmc"])
    sysd = F.make_system(F.MOLECULAR, n_orb=30, n_alpha=8, n_beta=8, h1=h1, eri=eri)
    qm = F.make_qmc(excit_gen=F.MOLECULAR, **q)
    caps = dict(main_capacity=1 << 28, spawn_capacity=1 << 27)
    say(f"[case] molecular D = {D}: FP64 run to iteration {T0}")
    fp = F.Context([sysd], [qm], F.SemiStoch(size=D, start_iteration=T0, precision=F.SS_FP64), graph=True, **caps)
    fp.step(T0)
    e0 = fp.estimators()
    shift, nprev, vary = fp.shift_state()
    keys, pops = fp.export()
    kd_fp, _ = fp.detspace()
    say(f"[case] {len(pops)} determinants, {e0['n_walkers_units'] / 256:.4g} walkers, shift {shift:.5f}, "
        f"varying {vary}")
    assert vary == 1 and len(kd_fp) == D
    sp = F.Context([sysd], [qm], F.SemiStoch(size=D, start_iteration=T0, precision=F.SS_SPLIT_BF16, check_period=50),
                   graph=True, **caps)
    sp.import_walkers(keys, pops, shift=shift, iteration=int(e0["iteration"]), vary=vary, n_prev=nprev)
    kd_sp, _ = sp.detspace()
    assert np.array_equal(kd_fp, kd_sp)
    say(f"[case] both runs: {N_ITER} iterations")
    fp.step(N_ITER)
    sp.step(N_ITER)
    hf, hs = fp.history(), sp.history()
    assert len(hf) == len(hs) == N_ITER
    ef, sf, kf = _energy(hf)
    es, ss_, ks = _energy(hs)
    errs = [h["ss_error"] for h in hs if h["ss_error"] > 0]
    bound = hs[-1]["ss_error_bound"]
    say(f"[case] FP64 {ef:.6f} +- {sf:.6f} (level {kf}), split {es:.6f} +- {ss_:.6f} (level {ks}); "
        f"split error ratio max {max(errs):.3e}, bound {bound:.3e}")
    assert errs and max(errs) <= bound
    assert abs(ef - es) <= 2.0 * math.sqrt(sf * sf + ss_ * ss_)
    # the runs separated: rounding differences change the stochastic dynamics
    assert any(a["n_walkers_units"] != b["n_walkers_units"] for a, b in zip(hf, hs))
    fp.close()
    sp.close()
