"""GPU walker lists and estimators against the oracle, bit for bit.

Given the same Philox keys every step of the iteration is deterministic and
order independent (integer populations, content-keyed random streams), so the
HIP path must reproduce the oracle's main list exactly after every iteration
and its estimators to the last bit (the projected-energy numerator is an exact
fixed-point sum on both sides).
"""
import numpy as np
import pytest

from gpu_helpers import (assert_same_estimators, assert_same_lists, gpu_context, oracle_qmc, oracle_system,
                         say, split_bound_check)
from paper_1811_11679_amd import synth, workloads

pytestmark = pytest.mark.gpu


def _compare_run(sysd, q, n_iter, every, ints=None, ss=None, main_cap=1 << 21, spawn_cap=1 << 21, tag=""):
    say(f"[case] {tag}: {n_iter} iterations, compare every {every}")
    ctx = gpu_context([sysd], [q], ints=ints, ss=ss, main_capacity=main_cap, spawn_capacity=spawn_cap)
    run = oracle_system(sysd, ints)
    orun = __import__("oracle.oracle", fromlist=["Run"]).Run(run, oracle_qmc(sysd, q, ss=ss))
    done = 0
    while done < n_iter:
        k = min(every, n_iter - done)
        ctx.step(k)
        orun.step(k)
        done += k
        assert_same_lists(ctx, orun, where=f"{tag} iteration {done}")
        hist = ctx.history()
        assert len(hist) == k
        assert_same_estimators(hist[-1], orun.estimators(), where=f"{tag} iteration {done}")
    say(f"[case] {tag}: final N_w units {orun.estimators()['n_walkers_units']}, "
        f"occupied {orun.estimators()['n_occupied']}")
    ctx.close()
    return orun.estimators()


def test_hubbard_ring_full_run_bitexact():
    w = workloads.HUBBARD8
    e = _compare_run(w["system"], w["qmc"], w["iterations"], 100, tag="hubbard8")
    assert e["vary_shift"] == 1


def test_hubbard_open_chain_odd_filling():
    sysd = dict(kind="hubbard", n_sites=7, periodic=0, t=1.0, U=2.5, n_alpha=3, n_beta=2)
    q = dict(tau=0.01, rng_seed=11, init_pop=200.0, target_population=3e3, initial_shift=-5.3)
    _compare_run(sysd, q, 300, 50, tag="hubbard7-open")


def test_ueg_two_word_keys_initiator_fixed_point():
    w = workloads.UEG14
    q = dict(w["qmc"], init_pop=3e3, target_population=1.5e4)
    _compare_run(w["system"], q, 300, 30, tag="ueg14-small", main_cap=1 << 23, spawn_cap=1 << 23)


def test_ueg_one_word_keys():
    sysd = dict(kind="ueg", rs=2.0, ecut_n2=3, n_alpha=5, n_beta=4)
    q = dict(tau=0.004, rng_seed=3, init_pop=5e3, target_population=5e4, initiator=1, initiator_threshold=2.0,
             fixed_point_bits=6, spawn_cutoff=0.25)
    _compare_run(sysd, q, 200, 25, tag="ueg9-w1")


def test_ueg_eight_word_keys():
    w = workloads.UEG54
    q = dict(w["qmc"], init_pop=2e3, target_population=1e9)
    _compare_run(w["system"], q, 30, 10, tag="ueg54-w8")


def test_molecular_heatbath():
    h1, eri = synth.molecular_integrals()
    w = workloads.MOL30
    q = dict(w["qmc"], init_pop=2e3, target_population=3e4)
    _compare_run(w["system"], q, 150, 15, ints=(h1, eri), tag="mol30")


def test_semistochastic_fp64_hubbard():
    w = workloads.HUBBARD8
    ss = dict(size=600, start_iteration=150)
    _compare_run(w["system"], w["qmc"], 500, 50, ss=ss, tag="hubbard8-ss")


def test_semistochastic_fp64_molecular_projection():
    h1, eri = synth.molecular_integrals()
    w = workloads.MOL30
    q = dict(w["qmc"], init_pop=2e3, target_population=3e4)
    ss = dict(size=200, start_iteration=40)
    say("[case] mol30-ss")
    ctx = gpu_context([w["system"]], [q], ints=(h1, eri), ss=ss)
    from oracle import oracle as O
    orun = O.Run(oracle_system(w["system"], (h1, eri)), oracle_qmc(w["system"], q, ss=ss))
    for it in range(4):
        ctx.step(20)
        orun.step(20)
        assert_same_lists(ctx, orun, where=f"mol30-ss block {it}")
        assert_same_estimators(ctx.estimators(), orun.estimators())
    kd, y = ctx.detspace()
    assert np.array_equal(kd, orun.detspace())
    assert np.array_equal(y, orun.last_projection())
    ctx.close()


def test_spawned_walkers_match_as_multisets():
    w = workloads.UEG14
    q = dict(w["qmc"], init_pop=2e4, target_population=1e9)
    from oracle import oracle as O
    orun = O.Run(oracle_system(w["system"]), oracle_qmc(w["system"], q))
    orun.step(60)
    keys, pops = orun.export()
    e = orun.estimators()
    say("[case] spawn multiset, imported state of", len(pops), "determinants")
    ctx = gpu_context([w["system"]], [q])
    ctx.import_walkers(keys, pops, shift=e["shift"], iteration=e["iteration"], vary=e["vary_shift"])
    orun2 = O.Run(oracle_system(w["system"]), oracle_qmc(w["system"], q))
    orun2.import_walkers(keys, pops, shift=e["shift"], iteration=e["iteration"], vary=e["vary_shift"])
    ctx.step(1)
    orun2.step(1)
    sg = ctx.spawns()
    so = orun2.spawns()
    tg = sorted(zip(map(tuple, sg[0].tolist()), sg[1].tolist(), sg[2].tolist()))
    to = sorted(zip(map(tuple, so[0].tolist()), so[1].tolist(), so[2].tolist()))
    assert len(tg) == len(to) and tg == to
    assert_same_lists(ctx, orun2, where="after import + 1")
    ctx.close()


def test_batched_replicas_match_independent_runs():
    sysd = dict(kind="ueg", rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)
    qs = [dict(tau=0.003, rng_seed=7, init_pop=3e3 * (r + 1), target_population=2e4 * (r + 1), initiator=1,
               initiator_threshold=3.0, fixed_point_bits=8, spawn_cutoff=0.1) for r in range(5)]
    say("[case] batched 5 replicas")
    ctx = gpu_context([sysd] * 5, qs, replicas=list(range(5)))
    from oracle import oracle as O
    runs = [O.Run(oracle_system(sysd), oracle_qmc(sysd, qs[r], replica=r)) for r in range(5)]
    for blk in range(6):
        ctx.step(20)
        for r in range(5):
            runs[r].step(20)
            assert_same_lists(ctx, runs[r], instance=r, where=f"replica {r} block {blk}")
            assert_same_estimators(ctx.estimators(r), runs[r].estimators(), where=f"replica {r}")
    ctx.close()


def test_batched_uneven_systems_same_width():
    # replicas of different rs and basis size (all W = 1) in one context
    sysds = [dict(kind="ueg", rs=rs, ecut_n2=ec, n_alpha=7, n_beta=7) for rs, ec in
             [(0.5, 2), (1.0, 3), (2.0, 2), (4.0, 3)]]
    qs = [dict(tau=0.002 * min(1.0, s["rs"] ** 2), rng_seed=7, init_pop=2e3, target_population=3e4,
               initiator=1, initiator_threshold=3.0, fixed_point_bits=8, spawn_cutoff=0.1) for s in sysds]
    say("[case] batched uneven systems")
    ctx = gpu_context(sysds, qs, replicas=[0, 1, 2, 3])
    from oracle import oracle as O
    runs = [O.Run(oracle_system(s), oracle_qmc(s, q, replica=r)) for r, (s, q) in enumerate(zip(sysds, qs))]
    for blk in range(4):
        ctx.step(25)
        for r in range(4):
            runs[r].step(25)
            assert_same_lists(ctx, runs[r], instance=r, where=f"uneven replica {r} block {blk}")
    ctx.close()


def test_capacity_overflow_rolls_back_to_iteration_start():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.UEG14
    q = dict(w["qmc"], init_pop=2e4, target_population=1e9)
    say("[case] spawn capacity overflow")
    ctx = gpu_context([w["system"]], [q], spawn_capacity=3000)
    from oracle import oracle as O
    orun = O.Run(oracle_system(w["system"]), oracle_qmc(w["system"], q))
    with pytest.raises(F.FqError) as ei:
        ctx.step(200)
    assert ei.value.code == F.FQ_ECAPACITY and "spawn capacity exceeded" in str(ei.value)
    t = ctx.estimators()["iteration"]
    orun.step(int(t))
    assert_same_lists(ctx, orun, where="state at the start of the failing iteration")
    ctx.close()


def test_empty_spawn_iterations_and_tiny_lists():
    # tiny time step: most iterations spawn nothing; one determinant to start
    sysd = dict(kind="hubbard", n_sites=4, periodic=1, t=1.0, U=1.0, n_alpha=1, n_beta=1)
    q = dict(tau=1e-4, rng_seed=5, init_pop=3.0, target_population=1e6)
    _compare_run(sysd, q, 60, 20, tag="tiny")


def test_segments_spanning_several_reduction_tiles():
    """Determinants that receive thousands of spawns in one iteration: the
    annihilation's segments of equal determinants span whole tiles of the
    segmented reduction (1024 spawns), so segment totals are assembled across
    tiles. A 6-site ring whose reference holds 2e5 integer walkers spawns
    ~2e4 times into each of its few neighbours."""
    sysd = dict(kind="hubbard", n_sites=6, periodic=1, t=1.0, U=4.0, n_alpha=3, n_beta=3)
    q = dict(tau=0.01, rng_seed=13, init_pop=2e5, target_population=1e9, initial_shift=-3.0)
    e = _compare_run(sysd, q, 12, 3, tag="long segments", main_cap=1 << 16, spawn_cap=1 << 22)
    assert e["n_spawned"] > 50 * e["n_spawn_events"]  # many spawns per distinct determinant


def test_export_import_roundtrip_and_resume():
    w = workloads.UEG14
    q = dict(w["qmc"], init_pop=2e4, target_population=1e9)
    say("[case] export/import resume")
    a = gpu_context([w["system"]], [q])
    a.step(30)
    keys, pops = a.export()
    e = a.estimators()
    b = gpu_context([w["system"]], [q])
    b.import_walkers(keys, pops, shift=e["shift"], iteration=e["iteration"], vary=e["vary_shift"])
    kb, pb = b.export()
    assert np.array_equal(kb, keys) and np.array_equal(pb, pops)
    a.step(20)
    b.step(20)
    ka, pa = a.export()
    kb, pb = b.export()
    assert np.array_equal(ka, kb) and np.array_equal(pa, pb)
    a.close()
    b.close()


def test_semistochastic_split_precision_error_within_bound():
    """BF16 x3 MFMA projection: at the first projected iteration the state is the
    oracle's, so the FP64 check equals the oracle's projection bit for bit and,
    row by row, the split result lies within the stated bound of it relative to
    sum_j |K_ij| |c_j| (K_DD from the oracle's matrix elements)."""
    h1, eri = synth.molecular_integrals()
    w = workloads.MOL30
    q = dict(w["qmc"], init_pop=2e3, target_population=3e4)
    ss = dict(size=300, start_iteration=30, precision=1, check_period=1)
    say("[case] mol30 split-precision projection")
    ctx = gpu_context([w["system"]], [q], ints=(h1, eri), ss=ss)
    from oracle import oracle as O
    osys = oracle_system(w["system"], (h1, eri))
    orun = O.Run(osys, oracle_qmc(w["system"], q, ss=ss))
    ctx.step(30)
    orun.step(30)
    start = orun.export()
    ctx.step(1)
    orun.step(1)
    kd, y = ctx.detspace()
    assert np.array_equal(kd, orun.detspace())
    yo = orun.last_projection()
    e = ctx.estimators()
    assert 0.0 < e["ss_error"] <= e["ss_error_bound"]
    ratio = split_bound_check(osys, kd, start, y, yo, e["ss_error_bound"])
    assert abs(ratio - e["ss_error"]) <= 1e-6 * e["ss_error"] + 1e-15
    say(f"[case] split projection: error ratio {ratio:.3e} (reported {e['ss_error']:.3e}), "
        f"bound {e['ss_error_bound']:.3e}")
    # the run continues in split precision with errors inside the bound
    ctx.step(50)
    hist = ctx.history()
    assert all(h["ss_error"] <= h["ss_error_bound"] for h in hist)
    ctx.close()


def test_tau_search_lowers_tau_identically():
    # a time step twice too large for the 19-plane-wave gas: the search lowers
    # it at the shift updates, on the GPU exactly as in the oracle
    sysd = dict(kind="ueg", rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)
    q = dict(tau=0.02, rng_seed=11, init_pop=3e3, target_population=2e4, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1, tau_search=1)
    e = _compare_run(sysd, q, 120, 20, tag="tau search ueg19")
    assert e["tau"] < 0.02 and e["spawn_ratio_max"] > 0.0
    assert e["tau"] * e["spawn_ratio_max"] <= 1.0 + 1e-15


def test_tau_search_per_replica():
    # three batched replicas of the gas at different densities, two with time
    # steps too large and one small enough to stay: each replica's search sees
    # only its own attempts and death steps, as one oracle run does (one
    # maximum for the context would lower the first replica's tau to the
    # densest gas's bound), and lowers only its own tau
    sysds = [dict(kind="ueg", rs=rs, ecut_n2=2, n_alpha=7, n_beta=7) for rs in (1.0, 2.0, 0.5)]
    taus = (0.02, 0.08, 0.002)
    qs = [dict(tau=taus[r], rng_seed=11 + r, init_pop=3e3, target_population=2e4, initiator=1,
               initiator_threshold=3.0, fixed_point_bits=8, spawn_cutoff=0.1, tau_search=1) for r in range(3)]
    say("[case] tau search, 3 batched replicas")
    ctx = gpu_context(sysds, qs, replicas=[0, 1, 2])
    from oracle import oracle as O
    runs = [O.Run(oracle_system(sysds[r]), oracle_qmc(sysds[r], qs[r], replica=r)) for r in range(3)]
    for blk in range(6):
        ctx.step(20)
        for r in range(3):
            runs[r].step(20)
            assert_same_lists(ctx, runs[r], instance=r, where=f"tau search replica {r} block {blk}")
            assert_same_estimators(ctx.estimators(r), runs[r].estimators(), where=f"tau search replica {r}")
    e = [runs[r].estimators() for r in range(3)]
    assert e[0]["tau"] < taus[0] and e[1]["tau"] < taus[1] and e[2]["tau"] == taus[2]
    assert e[0]["tau"] > 1.0 / e[2]["spawn_ratio_max"]
    for x in e:
        assert x["spawn_ratio_max"] > 0.0 and x["tau"] * x["spawn_ratio_max"] <= 1.0 + 1e-15
    ctx.close()
