"""The 54-electron gas at its full size, in the benchmark's launch configuration.

54 electrons in 251 plane waves (502 spin-orbitals, eight-word keys), about
1.8e8 determinants, the 8192-determinant space projected in split precision,
graph replay. One iteration is checked without re-running the list on the CPU
(the oracle cannot hold it): sampled parents outside the deterministic space
are re-run one by one by the oracle (a run holding only that parent draws the
same keyed random numbers), so their spawns must appear in the GPU's spawned
list and, when nothing spawns onto them, their new population must equal the
oracle's death step; the merged populations of sampled spawned-to determinants
outside the space must equal the oracle's death step of their own entry plus
every spawn the GPU sent to them, with the initiator rule for new ones; and
the population balance of the annihilation must hold for the whole list.
Members of the deterministic space are left out: their update is the split
projection, checked against its bound elsewhere.
"""
import numpy as np
import pytest

from gpu_helpers import say
from oracle import oracle as O
from paper_1811_11679_amd import workloads

pytestmark = pytest.mark.gpu

N_SAMPLE = 2000


def _find(sorted_keys, key):
    """Row of a key in an array sorted as unsigned big integers (last word most
    significant), or -1."""
    a, b = 0, len(sorted_keys)
    for w in range(sorted_keys.shape[1] - 1, -1, -1):
        col = sorted_keys[a:b, w]
        v = np.uint64(key[w])
        lo, hi = np.searchsorted(col, v, "left"), np.searchsorted(col, v, "right")
        if lo == hi:
            return -1
        a, b = a + lo, a + hi
    return int(a)


def _tup(k):
    return tuple(int(x) for x in k)


def _fingerprint(keys):
    """A 64-bit fingerprint of each W-word key (for grouping equal keys)."""
    h = np.zeros(len(keys), np.uint64)
    with np.errstate(over="ignore"):
        for w in range(keys.shape[1]):
            h = (h ^ keys[:, w]) * np.uint64(0x9E3779B97F4A7C15)
            h ^= h >> np.uint64(29)
    return h


def test_ueg54_full_size_iteration_sampled_against_oracle():
    from paper_1811_11679_amd import fciqmc as F
    w = workloads.UEG54
    s, q = w["system"], w["qmc"]
    start = 300
    say(f"[case] UEG54 full size, graph replay, D = {w['semistoch']['size']} split from iteration {start}: "
        f"400 iterations, then one checked")
    ss = F.SemiStoch(size=w["semistoch"]["size"], start_iteration=start, precision=F.SS_SPLIT_BF16, check_period=0)
    ctx = F.Context([F.make_system(F.UEG, rs=s["rs"], ecut_n2=s["ecut_n2"], n_alpha=s["n_alpha"], n_beta=s["n_beta"])],
                    [F.make_qmc(excit_gen=F.UEG, **q)], ss, main_capacity=330_000_000, spawn_capacity=200_000_000,
                    graph=True)
    assert ctx.W == 8
    for b in range(8):
        ctx.step(50)
        e = ctx.estimators()
        say(f"[case] iteration {e['iteration']}: {e['n_occupied']} determinants")
    e0 = ctx.estimators()
    shift, nprev, vary = ctx.shift_state()
    dkeys, _ = ctx.detspace()
    dset = {_tup(k) for k in dkeys}
    say("[case] exporting the list")
    k0, p0 = ctx.export()
    say(f"[case] {len(p0)} determinants, {e0['n_walkers_units'] / 256:.4g} walkers, shift {shift:.4f}")
    assert len(p0) > 100_000_000 and len(dset) == w["semistoch"]["size"]
    ctx.step(1)
    e1 = ctx.estimators()
    say("[case] one iteration done; exporting the list and the spawns")
    k1, p1 = ctx.export()
    sk, sa, si = ctx.spawns()
    say(f"[case] {len(sa)} spawns, {len(p1)} determinants after")
    # population balance over the whole list (the deterministic entries' change
    # is part of death_sum, the projection replacing their death step)
    assert int(p1.astype(np.int64).sum()) == e1["death_sum"] + e1["spawn_sum"] - e1["rejected_sum"]
    assert int(np.abs(p1.astype(np.int64)).sum()) == e1["n_walkers_units"] and len(p1) == e1["n_occupied"]
    assert int(sa.astype(np.int64).sum()) == e1["spawn_sum"] and len(sa) == e1["n_spawned"]
    rng = np.random.default_rng(5)
    for i in rng.integers(0, len(k1) - 1, 2000):
        assert _tup(k1[i][::-1]) < _tup(k1[i + 1][::-1])  # distinct, in key order

    osys = O.System.ueg(s["rs"], s["ecut_n2"], s["n_alpha"], s["n_beta"])
    oq = O.make_qmc(tau=q["tau"], seed=q["rng_seed"], init_pop=q["init_pop"], target_population=q["target_population"],
                    shift_period=q["shift_period"], shift_damping=q["shift_damping"], excit_gen=O.EXGEN_UEG,
                    initiator=1, initiator_threshold=q["initiator_threshold"], fixed_point_bits=8,
                    spawn_cutoff=q["spawn_cutoff"])
    it0 = int(e0["iteration"])

    def own_after_step(key, pop):
        run = O.Run(osys, oq)
        run.import_walkers(key[None, :], np.array([pop], np.int32), shift=shift, iteration=it0, vary=vary,
                           n_prev=nprev)
        run.step(1)
        kd, pd = run.export()
        return dict(zip((_tup(k) for k in kd), pd.tolist())).get(_tup(key), 0), run

    # spawns grouped by key through a fingerprint (keys are compared in full below)
    fp = _fingerprint(sk)
    so = np.argsort(fp)
    gfp, gk, ga, gi = fp[so], sk[so], sa[so], si[so]
    new = np.ones(len(gk), bool)
    new[1:] = gfp[1:] != gfp[:-1]
    g_lo = np.flatnonzero(new)
    g_hi = np.append(g_lo[1:], len(gk))
    say(f"[case] {len(g_lo)} distinct spawned determinants")

    def spawn_group(key):
        """[lo, hi) of the spawns onto key in the grouped arrays, or None"""
        f = _fingerprint(key[None, :])[0]
        g = int(np.searchsorted(g_lo, np.searchsorted(gfp, f), "right")) - 1
        if g < 0 or gfp[g_lo[g]] != f:
            return None
        lo, hi = g_lo[g], g_hi[g]
        assert np.all(gk[lo:hi] == key), "fingerprint collision"
        return lo, hi

    # 1. sampled parents outside the deterministic space
    wanted, deaths = {}, 0
    for i in rng.choice(len(p0), N_SAMPLE, replace=False):
        if _tup(k0[i]) in dset:
            continue
        own, run = own_after_step(k0[i], int(p0[i]))
        ok_, oa, oi = run.spawns()
        for kk, a, f in zip(ok_, oa.tolist(), oi.tolist()):
            if _tup(kk) not in dset:
                wanted.setdefault(_tup(kk), []).append((a, f))
        if spawn_group(k0[i]) is None:
            j = _find(k1, k0[i])
            assert (int(p1[j]) if j >= 0 else 0) == own, (i, own)
            deaths += 1
    n_checked = 0
    for kk, lst in wanted.items():
        r = spawn_group(np.array(kk, np.uint64))
        assert r is not None, kk
        pool = list(zip(ga[r[0]:r[1]].tolist(), gi[r[0]:r[1]].tolist()))
        for item in lst:
            assert item in pool, (kk, item)
            pool.remove(item)
            n_checked += 1
    say(f"[case] {n_checked} sampled spawns and {deaths} death steps identical to the oracle")
    assert n_checked > 100 and deaths > N_SAMPLE // 2

    # 2. merged populations of sampled spawned-to determinants: most spawns land
    # on unoccupied determinants, so the occupied ones are sampled on their own
    # (found through fingerprints of the old list, then compared in full)
    say("[case] finding spawned-to determinants that were occupied")
    fp0 = np.sort(_fingerprint(k0))
    gf = gfp[g_lo]
    pos = np.minimum(np.searchsorted(fp0, gf), len(fp0) - 1)
    occ_groups = np.flatnonzero(fp0[pos] == gf)
    del fp0
    occ_groups = occ_groups[~np.isin(gf[occ_groups], _fingerprint(dkeys))]  # not in the deterministic space
    say(f"[case] {len(occ_groups)} of them may have been occupied")
    picks = np.concatenate([rng.choice(len(g_lo), 300, replace=False),
                            rng.choice(occ_groups, min(150, len(occ_groups)), replace=False)])
    n_occ = n_new = n_rej = 0
    for g in picks:
        key = gk[g_lo[g]]
        if _tup(key) in dset:
            continue
        amps = ga[g_lo[g]:g_hi[g]].astype(np.int64)
        inits = gi[g_lo[g]:g_hi[g]]
        i0 = _find(k0, key)
        if i0 >= 0:
            own, _ = own_after_step(key, int(p0[i0]))
            want = own + int(amps.sum())
            n_occ += 1
        else:
            want = int(amps.sum()) if (inits.any() and int(amps.sum()) != 0) else 0
            n_new += int(want != 0)
            n_rej += int(want == 0)
        j = _find(k1, key)
        assert (int(p1[j]) if j >= 0 else 0) == want, (_tup(key), want)
    say(f"[case] merged populations of sampled spawned-to determinants identical: {n_occ} occupied, {n_new} created, "
        f"{n_rej} rejected or cancelled")
    assert n_occ + n_new + n_rej > 300 and n_occ >= min(50, len(occ_groups) // 2)
    ctx.close()
