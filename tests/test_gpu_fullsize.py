"""The benchmark workload at its full size, in the benchmark's launch configuration.

The 14-electron gas with the 1e7-walker target and the benchmark's list
capacities is run into its large-list regime (tens of millions of
determinants). One iteration is then checked without re-running the whole
list on the CPU:

* sampled outputs the oracle computes one by one: the spawns of sampled
  parents (an oracle run holding only that parent draws the same keyed random
  numbers) must all appear in the GPU's spawned list, and the new population
  of sampled parents that receive no spawns must equal the oracle's death step;
* merged populations of sampled spawned-to determinants: the oracle's death
  step of the determinant's own entry plus every spawn the GPU sent to it, and
  for determinants that were unoccupied the initiator rule (accepted iff some
  contribution came from an initiator); one iteration later the death step of
  sampled new determinants, which uses the diagonal element the GPU computed
  for them when they were created;
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


def _oracle_qmc(q):
    return O.make_qmc(tau=q["tau"], seed=q["rng_seed"], init_pop=q["init_pop"], target_population=q["target_population"],
                      shift_period=q["shift_period"], shift_damping=q["shift_damping"], excit_gen=O.EXGEN_UEG,
                      initiator=1, initiator_threshold=q["initiator_threshold"], fixed_point_bits=8,
                      spawn_cutoff=q["spawn_cutoff"])


def _own_after_step(osys, oq, key, pop, shift, it, vary, nprev):
    """The oracle's population of a lone determinant after one iteration: its
    death step (a lone entry receives no spawns)."""
    run = O.Run(osys, oq)
    run.import_walkers(key[None, :], np.array([pop], np.int32), shift=shift, iteration=it, vary=vary, n_prev=nprev)
    run.step(1)
    kd, pd = run.export()
    return dict(zip(_words_to_tuples(kd), pd.tolist())).get(tuple(int(x) for x in key), 0), run


def _spawn_groups(sk, sa, si):
    """Spawned records sorted by key, with [lo, hi) ranges per distinct key."""
    so = np.lexsort(sk.T)
    sk, sa, si = sk[so], sa[so], si[so]
    new = np.ones(len(sk), bool)
    new[1:] = np.any(sk[1:] != sk[:-1], axis=1)
    starts = np.flatnonzero(new)
    ends = np.append(starts[1:], len(sk))
    return sk, sa, si, starts, ends


def _full_size_iteration(pre_iterations, min_dets):
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.UEG14
    s, q = w["system"], w["qmc"]
    say(f"[case] UEG14 full size, graph replay: {pre_iterations} iterations, then two iterations checked")
    ctx = F.Context([F.make_system(F.UEG, rs=s["rs"], ecut_n2=s["ecut_n2"], n_alpha=s["n_alpha"], n_beta=s["n_beta"])],
                    [F.make_qmc(excit_gen=F.UEG, **q)], main_capacity=1 << 28, spawn_capacity=1 << 27, graph=True)
    ctx.step(pre_iterations)
    e0 = ctx.estimators()
    shift, nprev, vary = ctx.shift_state()
    k0, p0 = ctx.export()
    say(f"[case] {len(p0)} determinants, {e0['n_walkers_units'] / 256:.4g} walkers, shift {shift:.5f}")
    assert len(p0) > min_dets
    ctx.step(1)
    e1 = ctx.estimators()
    shift1, nprev1, vary1 = ctx.shift_state()
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

    osys = O.System.ueg(s["rs"], s["ecut_n2"], s["n_alpha"], s["n_beta"])
    oq = _oracle_qmc(q)
    it0 = int(e0["iteration"])
    gk, ga, gi, g_lo, g_hi = _spawn_groups(sk, sa, si)

    # 1. sampled parents against oracle runs that hold only that parent
    idx = rng.choice(len(p0), N_SAMPLE, replace=False)
    # the parent with the largest population (the reference) as well
    idx = np.concatenate([idx, [int(np.argmax(np.abs(p0)))]])
    wanted = {}
    deaths_checked = 0
    for i in idx:
        own, run = _own_after_step(osys, oq, k0[i], int(p0[i]), shift, it0, vary, nprev)
        ok_, oa, oi = run.spawns()
        for kk, a, f in zip(_words_to_tuples(ok_), oa.tolist(), oi.tolist()):
            wanted.setdefault(kk, []).append((a, f))
        parent = (int(k0[i, 0]), int(k0[i, 1]))
        if _find(gk, parent) < 0:
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

    # 2. merged populations of sampled spawned-to determinants
    groups = rng.choice(len(g_lo), N_SAMPLE, replace=False)
    n_occ = n_new = n_rej = 0
    new_children = []
    for g in groups:
        key = gk[g_lo[g]]
        amps = ga[g_lo[g]:g_hi[g]].astype(np.int64)
        inits = gi[g_lo[g]:g_hi[g]]
        i0 = _find(k0, key)
        if i0 >= 0:
            own, _ = _own_after_step(osys, oq, key, int(p0[i0]), shift, it0, vary, nprev)
            want = own + int(amps.sum())
            n_occ += 1
        else:
            accepted = bool(inits.any()) and int(amps.sum()) != 0
            want = int(amps.sum()) if accepted else 0
            n_new += int(accepted)
            n_rej += int(not accepted and int(amps.sum()) != 0)
        j = _find(k1, key)
        gpu = int(p1[j]) if j >= 0 else 0
        assert gpu == want, (tuple(int(x) for x in key), gpu, want)
        if i0 < 0 and j >= 0:
            new_children.append(j)
    say(f"[case] merged populations of {len(groups)} spawned-to determinants identical: {n_occ} occupied, "
        f"{n_new} created, {n_rej} refused by the initiator rule")
    assert n_occ > 0 and n_new > 0

    # 3. one more iteration: the death step of sampled new determinants (their
    # K_jj was computed on the GPU when they were created)
    extra = []
    for g in rng.choice(len(g_lo), 4 * N_SAMPLE, replace=False):
        key = gk[g_lo[g]]
        if _find(k0, key) < 0:
            j = _find(k1, key)
            if j >= 0:
                extra.append(j)
    new_children = sorted(set(new_children + extra))
    ctx.step(1)
    k2, p2 = ctx.export()
    sk2, sa2, si2 = ctx.spawns()
    hk, ha, hi_, h_lo, h_hi = _spawn_groups(sk2, sa2, si2)
    it1 = int(e1["iteration"])
    checked = 0
    for j in new_children:
        key = k1[j]
        own, _ = _own_after_step(osys, oq, key, int(p1[j]), shift1, it1, vary1, nprev1)
        g = _find(hk, key)  # first record of the key: the start of its group
        inc = 0
        if g >= 0:
            grp = int(np.searchsorted(h_lo, g))
            inc = int(ha[h_lo[grp]:h_hi[grp]].astype(np.int64).sum())
        jj = _find(k2, key)
        gpu = int(p2[jj]) if jj >= 0 else 0
        assert gpu == own + inc, (tuple(int(x) for x in key), gpu, own, inc)
        checked += 1
    say(f"[case] death steps of {checked} new determinants identical to the oracle")
    assert checked > 50
    ctx.close()


def test_ueg14_full_size_iteration_sampled_against_oracle():
    """Growth phase: the list still grows (shift not yet varied)."""
    _full_size_iteration(200, 10_000_000)


def test_ueg14_full_size_steady_state_sampled_against_oracle():
    """Steady state of the benchmark workload: population at target, shift settled."""
    _full_size_iteration(1500, 50_000_000)
