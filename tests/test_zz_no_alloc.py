"""The allocation-free set-up (fq_init_system_static) against fq_init_system.

A context whose workspace is the library's static device array must run the
same iterations as one on a caller-allocated workspace, bit for bit: walker
lists and every estimator. Two static contexts are made one after the other,
the second for a smaller system, so the second runs on an array that still
holds the first one's state. Oversized requests and a second live static
context on one device are refused.
"""
import numpy as np
import pytest

from paper_1811_11679_amd import fciqmc as F

FIELDS = ("iteration", "n_walkers_units", "n_occupied", "n_spawned", "ref_pop_units", "n_sign_flips",
          "n_spawn_events", "death_sum", "spawn_sum", "rejected_sum", "shift", "proj_numerator", "num_limbs")

CASES = [
    # 8-site ring, 4 + 4 electrons (4900 determinants)
    (dict(n_sites=8, periodic=1, t=1.0, U=4.0, n_alpha=4, n_beta=4),
     dict(tau=0.01, rng_seed=7, init_pop=500.0, target_population=1e4, shift_period=10, shift_damping=0.05,
          initial_shift=-4.0), 1 << 14, 1 << 16, 120),
    # a smaller input: 6-site ring, 3 + 3 electrons (400 determinants)
    (dict(n_sites=6, periodic=1, t=1.0, U=2.0, n_alpha=3, n_beta=3),
     dict(tau=0.01, rng_seed=11, init_pop=200.0, target_population=2e3, shift_period=10, shift_damping=0.05,
          initial_shift=-2.0), 1 << 12, 1 << 14, 120),
]


def _run(sysd, q, mc, sc, n, static):
    ctx = F.Context([F.make_system(F.HUBBARD, **sysd)], [F.make_qmc(excit_gen=1, **q)], main_capacity=mc,
                    spawn_capacity=sc, static_workspace=static)
    hist = []
    for _ in range(n // 20):
        ctx.step(20)
        hist += ctx.history()
    keys, pops = ctx.export()
    return ctx, keys, pops, hist


@pytest.mark.gpu
def test_static_workspace_matches_caller_workspace():
    for sysd, q, mc, sc, n in CASES:
        print(f"static workspace case: {sysd['n_sites']} sites, {n} iterations", flush=True)
        ref, kr, pr, hr = _run(sysd, q, mc, sc, n, static=False)
        ref.close()
        st, ks, ps, hs = _run(sysd, q, mc, sc, n, static=True)
        assert st.workspace is None
        # the other set-up entry point refuses while this context holds the array
        with pytest.raises(F.FqError) as ei:
            F.Context([F.make_system(F.HUBBARD, **sysd)], [F.make_qmc(excit_gen=1, **q)], main_capacity=mc,
                      spawn_capacity=sc, static_workspace=True)
        assert ei.value.code == F.FQ_ESTATE
        st.close()
        assert np.array_equal(kr, ks) and np.array_equal(pr, ps)
        assert len(hr) == len(hs) == n
        for a, b in zip(hr, hs):
            for f in FIELDS:
                assert a[f] == b[f], (f, a["iteration"], a[f], b[f])
        assert hs[-1]["n_walkers_units"] > 0


@pytest.mark.gpu
def test_static_workspace_refuses_oversized_capacity():
    sysd, q, _, _, _ = CASES[0]
    with pytest.raises(F.FqError) as ei:
        F.Context([F.make_system(F.HUBBARD, **sysd)], [F.make_qmc(excit_gen=1, **q)], main_capacity=1 << 22,
                  spawn_capacity=1 << 22, static_workspace=True)
    assert ei.value.code == F.FQ_ECAPACITY
    # nothing is held after the refusal: a fitting request succeeds
    ctx = F.Context([F.make_system(F.HUBBARD, **sysd)], [F.make_qmc(excit_gen=1, **q)], main_capacity=1 << 12,
                    spawn_capacity=1 << 14, static_workspace=True)
    ctx.step(10)
    assert ctx.estimators()["iteration"] == 10
    ctx.close()
