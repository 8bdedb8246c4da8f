"""The benchmark workload at its full size, in the benchmark's launch configuration.

The 14-electron gas with the 1e7-walker target and the benchmark's list
capacities is run into its large-list regime (tens of millions of
determinants). One iteration is then checked without re-running the whole
list on the CPU:

* sampled outputs the oracle computes one by one: the spawns of sampled
  parents (an oracle run holding only that parent draws the same keyed random
  numbers) must all appear in the GPU's spawned list, and the new population
  of sampled parents that receive no spawns must equal the oracle's death step;
* properties that hold at any size: the signed population balance of the
  annihilation, the walker count, the spawned amplitude sum, distinct and
  well-formed keys.
"""
import numpy as np
import pytest

from gpu_helpers import say
from oracle import oracle as O
from paper_1811_11679_amd import workloads

pytestmark = pytest.mark.gpu

N_SAMPLE = 300


def _words_to_tuples(keys):
    return [tuple(int(x) for x in k) for k in keys]


def _find(sorted_keys, key):
    """Row of a two-word key in an array sorted by (word 1, word 0), or -1."""
    hi = np.uint64(key[1])
    a, b = np.searchsorted(sorted_keys[:, 1], hi, "left"), np.searchsorted(sorted_keys[:, 1], hi, "right")
    if a == b:
        return -1
    j = a + np.searchsorted(sorted_keys[a:b, 0], np.uint64(key[0]))
    return int(j) if j < b and int(sorted_keys[j, 0]) == key[0] else -1


def test_ueg14_full_size_iteration_sampled_against_oracle():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.UEG14
    s, q = w["system"], w["qmc"]
    say("[case] UEG14 full size: 200 iterations, then one iteration checked")
    ctx = F.Context([F.make_system(F.UEG, rs=s["rs"], ecut_n2=s["ecut_n2"], n_alpha=s["n_alpha"], n_beta=s["n_beta"])],
                    [F.make_qmc(excit_gen=F.UEG, **q)], main_capacity=1 << 28, spawn_capacity=1 << 27)
    ctx.step(200)
    e0 = ctx.estimators()
    shift, nprev, vary = ctx.shift_state()
    k0, p0 = ctx.export()
    say(f"[case] {len(p0)} determinants, {e0['n_walkers_units'] / 256:.4g} walkers")
    assert len(p0) > 10_000_000
    ctx.step(1)
    e1 = ctx.estimators()
    k1, p1 = ctx.export()
    sk, sa, si = ctx.spawns()
    say(f"[case] {len(sa)} spawns, {len(p1)} determinants after")

    # properties of the new list and the spawned list
    assert int(p1.astype(np.int64).sum()) == e1["death_sum"] + e1["spawn_sum"] - e1["rejected_sum"]
    assert int(np.abs(p1.astype(np.int64)).sum()) == e1["n_walkers_units"]
    assert len(p1) == e1["n_occupied"]
    assert int(sa.astype(np.int64).sum()) == e1["spawn_sum"] and len(sa) == e1["n_spawned"]
    assert np.all(p1 != 0)
    order = np.lexsort(k1.T)  # most significant word last: the key order
    assert np.all(order == np.arange(len(order)))
    assert not np.any(np.all(k1[1:] == k1[:-1], axis=1))  # distinct keys
    alpha = np.uint64(0x5555555555555555)
    beta = np.uint64(0xAAAAAAAAAAAAAAAA)
    # 7 + 7 electrons in 114 spin-orbitals, on a spread of entries
    rng = np.random.default_rng(3)
    for i in rng.integers(0, len(k1), 5000):
        a = bin(int(k1[i, 0] & alpha)).count("1") + bin(int(k1[i, 1] & alpha)).count("1")
        b = bin(int(k1[i, 0] & beta)).count("1") + bin(int(k1[i, 1] & beta)).count("1")
        assert a == 7 and b == 7 and int(k1[i, 1]) >> (114 - 64) == 0

    # sampled parents against oracle runs that hold only that parent
    osys = O.System.ueg(s["rs"], s["ecut_n2"], s["n_alpha"], s["n_beta"])
    oq = O.make_qmc(tau=q["tau"], seed=q["rng_seed"], init_pop=q["init_pop"], target_population=q["target_population"],
                    shift_period=q["shift_period"], shift_damping=q["shift_damping"], excit_gen=O.EXGEN_UEG,
                    initiator=1, initiator_threshold=q["initiator_threshold"], fixed_point_bits=8,
                    spawn_cutoff=q["spawn_cutoff"])
    so = np.lexsort(sk.T)
    sk_sorted = sk[so]
    idx = rng.choice(len(p0), N_SAMPLE, replace=False)
    # the parent with the largest population (the reference) as well
    idx = np.concatenate([idx, [int(np.argmax(np.abs(p0)))]])
    wanted = {}
    deaths_checked = 0
    for i in idx:
        run = O.Run(osys, oq)
        run.import_walkers(k0[i:i + 1], p0[i:i + 1], shift=shift, iteration=int(e0["iteration"]), vary=vary,
                           n_prev=nprev)
        run.step(1)
        ok_, oa, oi = run.spawns()
        for kk, a, f in zip(_words_to_tuples(ok_), oa.tolist(), oi.tolist()):
            wanted.setdefault(kk, []).append((a, f))
        parent = (int(k0[i, 0]), int(k0[i, 1]))
        if _find(sk_sorted, parent) < 0:
            kd, pd = run.export()
            own = dict(zip(_words_to_tuples(kd), pd.tolist())).get(parent, 0)
            j = _find(k1, parent)
            gpu = int(p1[j]) if j >= 0 else 0
            assert gpu == own, (parent, gpu, own)
            deaths_checked += 1
    assert deaths_checked > N_SAMPLE // 2
    # every oracle spawn appears in the GPU's list (as a multiset per child)
    sel = np.isin(sk[:, 0], np.array([k[0] for k in wanted], np.uint64))
    have = {}
    for kk, a, f in zip(_words_to_tuples(sk[sel]), sa[sel].tolist(), si[sel].tolist()):
        have.setdefault(kk, []).append((a, f))
    n_checked = 0
    for kk, lst in wanted.items():
        pool = list(have.get(kk, []))
        for item in lst:
            assert item in pool, (kk, item)
            pool.remove(item)
            n_checked += 1
    say(f"[case] {n_checked} sampled spawns and {deaths_checked} death steps identical to the oracle")
    assert n_checked > 1000
    ctx.close()
