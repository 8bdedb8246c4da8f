"""One deterministic space shared by several replicas of one system.

FP64: the replicas' walker lists, estimators and deterministic spaces equal
the oracle's runs advanced with the same joint selection, bit for bit.
Split precision: K_DD C for all replicas is one BF16 x3 matrix product on
MFMA; at the first projected iteration the FP64 check equals the oracle's
projection exactly and the split result is within the stated bound.
"""
import numpy as np
import pytest

from gpu_helpers import (assert_same_estimators, assert_same_lists, gpu_context, oracle_qmc, oracle_system, say,
                         split_bound_check)
from oracle import oracle as O
from paper_1811_11679_amd import synth, workloads

pytestmark = pytest.mark.gpu


def test_shared_space_fp64_replicas_bitexact():
    w = workloads.HUBBARD8
    sysd = w["system"]
    R = 3
    qs = [dict(w["qmc"], init_pop=150.0 * (r + 1)) for r in range(R)]
    ss = dict(size=500, start_iteration=30, shared=1)
    say("[case] shared deterministic space, Hubbard 8 sites, 3 replicas, FP64")
    ctx = gpu_context([sysd] * R, qs, ss=ss, replicas=list(range(R)))
    runs = [O.Run(oracle_system(sysd), oracle_qmc(sysd, qs[r], replica=r, ss=ss)) for r in range(R)]
    for blk in range(6):
        ctx.step(10)
        O.step_shared(runs, 10)
        for r in range(R):
            assert_same_lists(ctx, runs[r], instance=r, where=f"shared replica {r} block {blk}")
            assert_same_estimators(ctx.estimators(r), runs[r].estimators(), where=f"shared replica {r}")
    for r in range(R):
        kd, y = ctx.detspace(r)
        assert np.array_equal(kd, runs[r].detspace())
        assert np.array_equal(y, runs[r].last_projection())
    ctx.close()


def test_shared_space_split_precision_gemm_within_bound():
    h1, eri = synth.molecular_integrals()
    w = workloads.MOL30
    R = 5
    qs = [dict(w["qmc"], init_pop=1e3 * (r + 1), target_population=3e4) for r in range(R)]
    ss = dict(size=200, start_iteration=30, precision=1, check_period=1, shared=1)
    say("[case] shared deterministic space, molecular, 5 replicas, split precision")
    ctx = gpu_context([w["system"]] * R, qs, ints=(h1, eri), ss=ss, replicas=list(range(R)))
    osys = oracle_system(w["system"], (h1, eri))
    runs = [O.Run(osys, oracle_qmc(w["system"], qs[r], replica=r, ss=ss)) for r in range(R)]
    ctx.step(30)
    O.step_shared(runs, 30)
    starts = [r.export() for r in runs]  # includes the members added with n = 0
    ctx.step(1)
    O.step_shared(runs, 1)
    for r in range(R):
        kd, y = ctx.detspace(r)
        assert np.array_equal(kd, runs[r].detspace())
        yo = runs[r].last_projection()
        e = ctx.estimators(r)
        assert 0.0 < e["ss_error"] <= e["ss_error_bound"]
        ratio = split_bound_check(osys, kd, starts[r], y, yo, e["ss_error_bound"])
        say(f"[case] replica {r}: error ratio {ratio:.3e} (reported {e['ss_error']:.3e}), "
            f"bound {e['ss_error_bound']:.3e}")
        assert abs(ratio - e["ss_error"]) <= 1e-6 * e["ss_error"] + 1e-15
    ctx.step(30)
    for r in range(R):
        assert all(h["ss_error"] <= h["ss_error_bound"] for h in ctx.history(r))
    ctx.close()
