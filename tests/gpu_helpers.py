"""Builds matching GPU contexts and oracle runs from one parameter set."""
import sys

import numpy as np

from oracle import oracle as O
from paper_1811_11679_amd import synth

KIND = {"hubbard": 1, "ueg": 2, "molecular": 3}


def oracle_system(sysd, ints=None):
    k = sysd["kind"]
    if k == "hubbard":
        return O.System.hubbard(sysd["n_sites"], bool(sysd.get("periodic", 1)), sysd.get("t", 1.0),
                                sysd.get("U", 0.0), sysd["n_alpha"], sysd["n_beta"])
    if k == "ueg":
        return O.System.ueg(sysd["rs"], sysd["ecut_n2"], sysd["n_alpha"], sysd["n_beta"])
    h1, eri = ints
    return O.System.molecular(h1, eri, sysd["n_alpha"], sysd["n_beta"])


def oracle_qmc(sysd, q, replica=0, ss=None):
    k = KIND[sysd["kind"]]
    return O.make_qmc(tau=q["tau"], seed=q.get("rng_seed", 7), replica_id=replica, init_pop=q["init_pop"],
                      target_population=q["target_population"], shift_period=q.get("shift_period", 10),
                      shift_damping=q.get("shift_damping", 0.05), initial_shift=q.get("initial_shift", 0.0),
                      excit_gen=k, p_single=q.get("p_single", 0.1), initiator=q.get("initiator", 0),
                      initiator_threshold=q.get("initiator_threshold", 3.0),
                      fixed_point_bits=q.get("fixed_point_bits", 0), spawn_cutoff=q.get("spawn_cutoff", 0.0),
                      ss_size=ss["size"] if ss else 0, ss_start_iteration=ss["start_iteration"] if ss else 0,
                      ss_shared=ss.get("shared", 0) if ss else 0, tau_search=q.get("tau_search", 0))


def gpu_context(sysds, qs, ints=None, ss=None, main_capacity=1 << 21, spawn_capacity=1 << 21,
                replicas=None, graph=False):
    from paper_1811_11679_amd import fciqmc as F
    systems, qmcs = [], []
    for i, (sysd, q) in enumerate(zip(sysds, qs)):
        k = KIND[sysd["kind"]]
        kw = {x: v for x, v in sysd.items() if x != "kind"}
        if k == 3:
            kw["h1"], kw["eri"] = ints
        systems.append(F.make_system(k, **kw))
        qq = dict(q)
        qq["excit_gen"] = k
        qq["replica_id"] = replicas[i] if replicas else 0
        qmcs.append(F.make_qmc(**qq))
    sso = None
    if ss:
        sso = F.SemiStoch(size=ss["size"], start_iteration=ss["start_iteration"],
                          precision=ss.get("precision", F.SS_FP64), check_period=ss.get("check_period", 0),
                          shared=ss.get("shared", 0))
    return F.Context(systems, qmcs, sso, main_capacity=main_capacity, spawn_capacity=spawn_capacity, graph=graph)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_same_lists(ctx, run, instance=0, where=""):
    kg, pg = ctx.export(instance)
    ko, po = run.export()
    assert kg.shape == ko.shape, f"{where}: {kg.shape} vs {ko.shape} determinants"
    assert np.array_equal(kg, ko), f"{where}: keys differ"
    if not np.array_equal(pg, po):
        bad = np.nonzero(pg != po)[0]
        raise AssertionError(f"{where}: {len(bad)} populations differ, first {pg[bad[:5]]} vs {po[bad[:5]]}")


FIELDS = ("iteration", "n_walkers_units", "n_occupied", "ref_pop_units", "n_spawned", "n_spawn_events",
          "death_sum", "spawn_sum", "rejected_sum", "n_rejected_units", "n_sign_flips", "vary_shift",
          "num_limbs", "pair_limbs", "n_cluster_spawns", "shift", "proj_numerator", "tau", "spawn_ratio_max")


def assert_same_estimators(eg, eo, where=""):
    for f in FIELDS:
        assert eg[f] == eo[f], f"{where}: estimator {f}: gpu {eg[f]} vs oracle {eo[f]}"
    pe, po = eg["proj_energy"], eo["proj_energy"]
    assert (np.isnan(pe) and np.isnan(po)) or pe == po, f"{where}: proj_energy {pe} vs {po}"


def split_bound_check(system, dkeys, start_state, y_split, y_fp64, bound):
    """Per row: |y_i - y_i(FP64)| <= bound * sum_j |K_ij| |c_j|, with K_DD from the
    oracle's matrix elements and c the populations the projection read."""
    keys, pops = start_state
    cur = {tuple(int(x) for x in k): int(p) for k, p in zip(keys, pops)}
    dl = [tuple(int(x) for x in k) for k in dkeys]
    c = np.array([cur.get(k, 0) for k in dl], float)
    h00 = system.H00
    K = np.array([[system.diag(np.array(a, np.uint64)) - h00 if i == j else
                   system.hij(np.array(a, np.uint64), np.array(b, np.uint64))
                   for j, b in enumerate(dl)] for i, a in enumerate(dl)])
    scale = np.abs(K) @ np.abs(c)
    err = np.abs(y_split - y_fp64)
    ok = scale > 0
    ratio = np.max(err[ok] / scale[ok])
    assert ratio <= bound, (ratio, bound)
    assert np.all(err[~ok] == 0)
    return ratio
