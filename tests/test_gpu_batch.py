"""Batching: graph replay, launch geometry, tile shapes and mixed-width
batches, all bit-exact.

Replaying a captured block of iterations, changing the number of blocks or the
tile shapes of the persistent kernels and spreading instances over several
contexts change how the work is scheduled, never what is computed: every case
below must give the oracle's walker lists and estimators to the last bit.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same_estimators, assert_same_lists, gpu_context, oracle_qmc, oracle_system, say
from oracle import oracle as O
from paper_1811_11679_amd import workloads
from paper_1811_11679_amd.fciqmc import TILE_VARIANTS as F_TILE_VARIANTS

pytestmark = pytest.mark.gpu


def _oracle_run(sysd, q, replica=0):
    return O.Run(oracle_system(sysd), oracle_qmc(sysd, q, replica=replica))


def test_graph_replay_matches_oracle_every_replay():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.HUBBARD8
    sysd, q = w["system"], w["qmc"]
    say("[case] graph replay hubbard8")
    ctx = F.Context([F.make_system(F.HUBBARD, **{k: v for k, v in sysd.items() if k != "kind"})],
                    [F.make_qmc(excit_gen=F.HUBBARD, **q)], main_capacity=1 << 21, spawn_capacity=1 << 21,
                    graph=True)
    run = _oracle_run(sysd, q)
    # aligned blocks replay the graphs of both list parities; the odd step
    # counts in between run directly and shift the phase of later blocks
    plan = [10, 10, 10, 7, 3, 10, 20, 5, 5, 10, 30, 13, 17, 10]
    done = 0
    for k in plan:
        ctx.step(k)
        run.step(k)
        done += k
        assert_same_lists(ctx, run, where=f"graph replay, iteration {done}")
        assert_same_estimators(ctx.estimators(), run.estimators(), where=f"graph replay, iteration {done}")
    ctx.close()


def test_launch_geometry_does_not_change_results():
    w = workloads.UEG14
    q = dict(w["qmc"], init_pop=3e3, target_population=1.5e4)
    say("[case] odd launch geometry ueg14-small")
    ctx = gpu_context([w["system"]], [q], main_capacity=1 << 23, spawn_capacity=1 << 23)
    ctx.set_launch({"spawn": 7, "merge": 3, "sort": 5, "reduce": 1, "new_diag": 2})
    assert ctx.get_launch() == {"spawn": 7, "merge": 3, "sort": 5, "reduce": 1, "new_diag": 2}
    run = _oracle_run(w["system"], q)
    for blk in range(4):
        ctx.step(25)
        run.step(25)
        assert_same_lists(ctx, run, where=f"odd geometry block {blk}")
        assert_same_estimators(ctx.estimators(), run.estimators())
    ctx.set_launch({"spawn": 4096, "merge": 4096, "sort": 4096, "reduce": 4096, "new_diag": 4096})
    ctx.step(25)
    run.step(25)
    assert_same_lists(ctx, run, where="large geometry")
    ctx.close()


def test_autotuner_keeps_the_run_exact():
    from paper_1811_11679_amd import autotune
    sysd = dict(kind="ueg", rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)
    q = dict(tau=0.003, rng_seed=7, init_pop=3e3, target_population=2e4, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1)
    say("[case] autotune ueg19")
    ctx = gpu_context([sysd], [q])
    run = _oracle_run(sysd, q)
    best = autotune.tune(ctx, iters=2, kernels=["merge", "sort"], log=say)
    n = int(ctx.estimators()["iteration"])
    tiles = best.pop("tiles")
    assert set(best) == {"spawn", "merge", "sort", "reduce", "new_diag"} and all(v > 0 for v in best.values())
    assert all(tiles[k] in F_TILE_VARIANTS[k] for k in tiles) and tiles == ctx.get_tiles()
    run.step(n)
    assert_same_lists(ctx, run, where=f"after autotuning ({n} iterations)")
    ctx.step(20)
    run.step(20)
    assert_same_lists(ctx, run, where="after autotuning + 20")
    ctx.close()


def test_every_tile_variant_matches_the_oracle():
    """Each compiled tile shape (spawning attempts, merge positions, radix-sort
    keys per thread) gives the oracle's walker lists: one-word Hubbard keys,
    two-word electron-gas keys (initiator, fixed point) and a batched pair of
    electron-gas replicas; the shape changes between blocks of iterations."""
    from paper_1811_11679_amd import fciqmc as F
    cases = [
        ([dict(kind="hubbard", n_sites=8, periodic=1, t=1.0, U=4.0, n_alpha=4, n_beta=4)],
         [dict(tau=0.01, rng_seed=7, init_pop=500.0, target_population=1e4, initial_shift=-4.0)]),
        ([dict(kind="ueg", rs=1.0, ecut_n2=5, n_alpha=7, n_beta=7)],
         [dict(tau=0.002, rng_seed=7, init_pop=3e3, target_population=3e4, initiator=1, initiator_threshold=3.0,
               fixed_point_bits=8, spawn_cutoff=0.1)]),
        ([dict(kind="ueg", rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)] * 2,
         [dict(tau=0.003, rng_seed=7, init_pop=2e3 * (r + 1), target_population=2e4, initiator=1,
               initiator_threshold=3.0, fixed_point_bits=8, spawn_cutoff=0.1, replica_id=r) for r in range(2)]),
    ]
    for sysds, qs in cases:
        say(f"[case] tile variants: {sysds[0]['kind']} x {len(sysds)}")
        ctx = gpu_context(sysds, qs, replicas=list(range(len(qs))) if len(qs) > 1 else None)
        runs = [_oracle_run(sysds[r], qs[r], replica=r) for r in range(len(qs))]
        ctx.step(30)
        for r in runs:
            r.step(30)
        for knob in F.TILE_KNOBS:
            for v in F.TILE_VARIANTS[knob]:
                ctx.set_tiles({knob: v})
                ctx.step(10)
                for i, r in enumerate(runs):
                    r.step(10)
                    assert_same_lists(ctx, r, instance=i, where=f"{knob} = {v}, instance {i}")
                    assert_same_estimators(ctx.estimators(i), r.estimators(), where=f"{knob} = {v}")
            ctx.set_tiles({knob: {"spawn_items": 4, "merge_items": 2, "sort_items": 12}[knob]})
        with pytest.raises(F.FqError):
            ctx.set_tiles({"merge_items": 3})
        ctx.close()


def test_mixed_width_batch_matches_plain_runs_and_oracle():
    from paper_1811_11679_amd import batch as B
    # electron-gas instances of three key widths (19 and 27 plane waves: one
    # word, 57: two words, 123: four words), uneven targets, distinct streams
    specs = [(1.0, 2, 3e3), (2.0, 5, 2e3), (0.5, 3, 4e3), (4.0, 9, 1.5e3), (1.0, 5, 2.5e3), (2.0, 2, 1e3)]
    inst = []
    for r, (rs, ec, tgt) in enumerate(specs):
        sysd = dict(kind="ueg", rs=rs, ecut_n2=ec, n_alpha=7, n_beta=7)
        q = dict(tau=0.002 * min(1.0, rs * rs), rng_seed=7, init_pop=tgt / 10, target_population=tgt, initiator=1,
                 initiator_threshold=3.0, fixed_point_bits=8, spawn_cutoff=0.1, replica_id=r)
        inst.append((sysd, q))
    say("[case] mixed-width batch of 6")
    bt = B.Batch(inst, capacity=lambda m: (1 << 22, 1 << 21))
    assert len(bt.contexts) == 3
    runs = [_oracle_run(s, q, replica=r) for r, (s, q) in enumerate(inst)]
    for blk in range(3):
        bt.step(20)
        for r in range(len(inst)):
            runs[r].step(20)
            g, slot = bt.where[r]
            assert_same_lists(bt.contexts[g], runs[r], instance=slot, where=f"batch instance {r} block {blk}")
            assert_same_estimators(bt.estimators(r), runs[r].estimators(), where=f"batch instance {r}")
    # a plain context of instance 3 continued from the batch's exported state
    # stays identical to the batch
    from gpu_helpers import gpu_context as gc
    s3, q3 = inst[3]
    keys, pops = bt.export(3)
    e = bt.estimators(3)
    sh, nprev, vary = bt.shift_state(3)
    plain = gc([s3], [{k: v for k, v in q3.items() if k != "replica_id"}], replicas=[3])
    plain.import_walkers(keys, pops, shift=sh, iteration=e["iteration"], vary=vary, n_prev=nprev)
    plain.step(30)
    bt.step(30)
    kp, pp = plain.export()
    kb, pb = bt.export(3)
    assert np.array_equal(kp, kb) and np.array_equal(pp, pb)
    assert_same_estimators(plain.estimators(), bt.estimators(3), where="plain continuation of instance 3")
    plain.close()
    bt.close()


def test_graph_replay_with_tau_search_matches_oracle():
    # the lowered time step reaches the captured kernels through device memory
    from paper_1811_11679_amd import fciqmc as F
    sysd = dict(kind="ueg", rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)
    q = dict(tau=0.02, rng_seed=11, init_pop=3e3, target_population=2e4, initiator=1, initiator_threshold=3.0,
             fixed_point_bits=8, spawn_cutoff=0.1, tau_search=1)
    say("[case] graph replay with tau search ueg19")
    ctx = F.Context([F.make_system(F.UEG, rs=1.0, ecut_n2=2, n_alpha=7, n_beta=7)],
                    [F.make_qmc(excit_gen=F.UEG, **q)], main_capacity=1 << 21, spawn_capacity=1 << 21, graph=True)
    run = _oracle_run(sysd, q)
    for k in (10, 10, 7, 3, 20, 30):
        ctx.step(k)
        run.step(k)
        assert_same_lists(ctx, run, where="graph replay with tau search")
        assert_same_estimators(ctx.estimators(), run.estimators(), where="graph replay with tau search")
    assert ctx.estimators()["tau"] < 0.02
    ctx.close()


def test_batch64_workload_one_instance_per_key_width_against_oracle():
    """The 64-instance batched electron-gas workload at its full size (three
    contexts: one-, two- and four-word keys). After 300 batched iterations, the
    smallest instance of each context is exported and continued by the oracle
    from that state for 20 iterations while the whole batch advances: its list
    and estimators stay identical to the oracle's."""
    from paper_1811_11679_amd import batch as B
    import bench

    inst = workloads.batch64()
    bt = B.Batch(inst, capacity=bench.batch_capacity(inst))
    say(f"[case] batch64: {len(inst)} instances in {len(bt.contexts)} contexts "
        f"(key words {[c.W for c in bt.contexts]})")
    assert sorted(c.W for c in bt.contexts) == [1, 2, 4]
    bt.step(300)
    checked = []
    for g, members in enumerate(bt.groups):
        i = min(members, key=lambda m: inst[m][1]["target_population"])
        sysd, q = inst[i]
        keys, pops = bt.export(i)
        shift, nprev, vary = bt.shift_state(i)
        e = bt.estimators(i)
        run = _oracle_run(sysd, q, replica=q["replica_id"])
        run.import_walkers(keys, pops, shift=shift, iteration=int(e["iteration"]), vary=vary, n_prev=nprev)
        checked.append((i, run))
        say(f"[case] instance {i}: {len(pops)} determinants, {e['n_walkers_units'] / 256:.4g} walkers, "
            f"key words {bt.contexts[g].W}")
    bt.step(20)
    for i, run in checked:
        run.step(20)
        g, slot = bt.where[i]
        assert_same_lists(bt.contexts[g], run, instance=slot, where=f"batch64 instance {i}")
        assert_same_estimators(bt.estimators(i), run.estimators(), where=f"batch64 instance {i}")
    bt.close()
