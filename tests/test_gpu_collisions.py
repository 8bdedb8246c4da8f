"""Hash collisions: many determinants on one sort key.

With only the top bits of each determinant's hash in its sort key, the main
list and every spawned list hold runs of equal sort keys with different
determinants, as a genuine 64-bit hash collision would. The annihilation
(Sec. 2.4) must still combine exactly the walkers of each determinant: the
merge breaks ties by the determinant, the collision fix-up puts every mixed
run of the spawned list in determinant order and the reduction is redone.
Two instances share a context (replica id in the top sort-key bit); each must
equal its own oracle run to the last bit. The random streams are keyed by the
full hash, so the dynamics do not change; only the list order does, and the
lists are compared in determinant order.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same_estimators, gpu_context, oracle_qmc, oracle_system, say
from oracle import oracle as O
from paper_1811_11679_amd import workloads

pytestmark = pytest.mark.gpu

UEG_SMALL = dict(system=workloads.UEG14["system"],
                 qmc=dict(workloads.UEG14["qmc"], init_pop=3e3, target_population=1.5e4))


def _by_key(keys, pops):
    o = np.lexsort(keys.T)
    return keys[o], pops[o]


def _masked_sort_keys(keys, bits, replica):
    """Sort keys as the truncated ordering defines them: replica bit on top,
    the top `bits` bits of the hash below it (two instances: one replica bit)."""
    mask = ((1 << 64) - 1) ^ ((1 << (64 - bits)) - 1)
    out = []
    for k in keys:
        h = O.hash64([int(x) for x in k]) & mask
        out.append((replica << 63) | (h >> 1))
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("case,bits,iters", [("hubbard8", 8, 6), ("ueg14_small", 12, 5)])
def test_truncated_sort_keys_match_oracle(case, bits, iters):
    w = workloads.HUBBARD8 if case == "hubbard8" else UEG_SMALL
    sysd, q = w["system"], w["qmc"]
    say(f"[case] {case}: sort keys from the top {bits} hash bits, two instances")
    ctx = gpu_context([sysd, sysd], [q, q], replicas=[0, 1], main_capacity=1 << 21, spawn_capacity=1 << 21)
    ctx.set_sort_key_bits(bits)
    runs = [O.Run(oracle_system(sysd), oracle_qmc(sysd, q, replica=r)) for r in (0, 1)]
    ties_seen = 0
    for blk in range(iters):
        ctx.step(10)
        for r in (0, 1):
            runs[r].step(10)
            kg, pg = ctx.export(r)
            ko, po = runs[r].export()
            # determinants that share a truncated sort key with another one
            # (adjacent in the device list, which is ordered by sort key)
            sk = _masked_sort_keys(kg, bits, r)
            ties_seen += len(sk) - len(np.unique(sk))
            kg, pg = _by_key(kg, pg)
            ko, po = _by_key(ko, po)
            assert np.array_equal(kg, ko), f"{case} instance {r} block {blk}: determinants differ"
            assert np.array_equal(pg, po), f"{case} instance {r} block {blk}: populations differ"
            assert_same_estimators(ctx.estimators(r), runs[r].estimators(), where=f"{case} instance {r} block {blk}")
    say(f"[case] {case}: {ties_seen} main-list entries shared a sort key with another determinant")
    assert ties_seen > 100
    ctx.close()


def test_too_many_determinants_on_one_sort_key_is_refused():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.HUBBARD8
    sysd, q = w["system"], w["qmc"]
    say("[case] hubbard8: one hash bit in the sort key (error path)")
    ctx = gpu_context([sysd, sysd], [q, q], replicas=[0, 1], main_capacity=1 << 21, spawn_capacity=1 << 21)
    ctx.set_sort_key_bits(1)
    with pytest.raises(F.FqError, match="share one sort key") as ei:
        ctx.step(200)
    assert ei.value.code == F.FQ_ESTATE
    # the context is left at the start of the failing iteration
    t = int(ctx.estimators(0)["iteration"])
    for r in (0, 1):
        run = O.Run(oracle_system(sysd), oracle_qmc(sysd, q, replica=r))
        run.step(t)
        kg, pg = _by_key(*ctx.export(r))
        ko, po = _by_key(*run.export())
        assert np.array_equal(kg, ko) and np.array_equal(pg, po), f"instance {r} after the refused iteration {t + 1}"
    say(f"[case] refused at iteration {t + 1}, state of iteration {t} kept")
    ctx.close()


def test_sort_key_truncation_argument_checks():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.HUBBARD8
    sysd, q = w["system"], w["qmc"]
    one = gpu_context([sysd], [q])
    with pytest.raises(F.FqError, match="two or more instances"):
        one.set_sort_key_bits(8)
    one.close()
    two = gpu_context([sysd, sysd], [q, q], replicas=[0, 1])
    for bad in (0, 65):
        with pytest.raises(F.FqError):
            two.set_sort_key_bits(bad)
    two.set_sort_key_bits(64)  # the full hash: the default ordering
    two.close()
