#!/usr/bin/env python
"""FCIQMC iteration throughput on one MI355X.

Default workload: initiator FCIQMC on the 3D uniform electron gas, 14
electrons (7 + 7), rs = 1, 57 plane waves (114 spin-orbitals, two-word keys),
Coulomb 4 pi / (L^3 k^2), real weights in 1/256 units, spawn cutoff 0.1,
initiator threshold 3, dtau = 0.002, target 1e7 walkers, shift varied every 10
iterations with damping 0.05; synthetic (the system is defined by its
parameters). The workload runs 5000 iterations and times the last 1000: the
first 4000 (equilibration, part of the workload) bring the population to its
target and let the shift settle; --warmup adds iterations after them and
--steps sets how many are timed.

One step = one whole projector iteration: spawning, radix sort, segmented
reduction, merge with death/initiator rule, estimators and the host shift
update. The timed window is replayed from captured HIP graphs (one per block of
iterations between shift updates) and bracketed by one pair of HIP events on
the context's stream plus device synchronisation; per-kernel durations come
from an equally long window right after it with an event around every launch
(events inside a captured graph record no elapsed time), at the same steady
state. A rocprofv3 run with --selected-regions profiles exactly those two
windows (roctxProfilerResume / roctxProfilerPause around them).

Prints one JSON line: walker updates/s = sum over the timed iterations of the
walker population at the start of each iteration, divided by the wall time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker updates/s per FCIQMC iteration, plain vs batched; annihilation HBM GB/s"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(hist_prev, hist, W, ds_active=False, instances=1, ccmc=None):
    """Bytes each kernel must move per iteration (reads + writes of the data it
    owns). The deterministic slot of a main entry (4 bytes) is read and written
    only while a deterministic space is active; its sort key (8 bytes) is
    stored when several instances share the list or keys are longer than two
    words (else it is the key's hash, recomputed)."""
    out = {}
    nm, nm2 = hist_prev["n_occupied"], hist["n_occupied"]
    ns, nu = hist["n_spawned"], hist["n_spawn_events"]
    kb = 8 * W
    ds = 4 if ds_active else 0
    sk = 8 if instances > 1 or W > 2 else 0
    # spawn: parent key, sort key, population, slot and attempt offset read;
    # per spawn its sort key and record (key words, amplitude | initiator flag)
    out["spawn"] = nm * (kb + sk + 4 + ds + 8) + ns * (8 + kb + 8)
    out["sort_pass0"] = ns * (8 + 8 + 4)
    for p in range(1, 8):
        out[f"sort_pass{p}"] = ns * (8 + 4) * 2
    out["sort_hist"] = ns * 8
    out["reduce"] = ns * (8 + 4 + kb + 8) + nu * (8 + kb + 8 + 4)
    # output: skey, key, pop, kdiag, slot, attempt offset and the new-determinant flag
    out["merge"] = nm * (sk + kb + 4 + 8 + ds) + nu * (8 + kb + 8 + 4) + nm2 * (sk + kb + 4 + 8 + ds + 8 + 1)
    out["new_diag"] = nm2 * 8
    if ccmc is not None:
        # CCMC (ccmc = (truncation, electrons, b)): the prefix scan reads key and
        # population and writes 8 bytes per entry; each of the n_c selections
        # reads the key and population of s excitors (s of expected value
        # sum_s p(s) s) and each composite record is written as for a spawn
        trunc, nel, b = ccmc
        smax = min(trunc + 2, nel)
        ps = {sz: 2.0 ** -(sz - 1) for sz in range(2, smax)}
        ps[smax] = 2.0 ** -(smax - 2)
        s_mean = sum(sz * p for sz, p in ps.items())
        nex = hist_prev["n_walkers_units"] - abs(hist_prev["ref_pop_units"])
        nc = -(-nex // (1 << b))
        out["ccmc_clusters"] = nm * (kb + 4 + 8) + nc * s_mean * (kb + 4) + hist["n_cluster_spawns"] * (8 + kb + 8)
        out["ccmc_pairs"] = nm2 * (kb + 4)
    return out


def kernel_sources_sha256():
    """SHA-256 over the device sources (the .hip files and the headers they
    include, in name order): what HBM counters of the kernels depend on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1811_11679_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of the
    workload, if the kernel sources are the ones it was measured on (else None)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel_sources_sha256() != rec.get("source_sha256"):
        return None
    k = rec["kernels"].get(kernel)
    return None if k is None else k["bytes_per_launch"]


class ProfilerRegion:
    """roctxProfilerResume(0) / roctxProfilerPause(0): under `rocprofv3
    --selected-regions` only what runs between them is traced or counted. No-op
    without the profiler (or without the roctx library)."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so", "/opt/rocm/lib/librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.lib is not None:
            # roctx_thread_id_t: 64 bits; 0 = every thread of the process
            for f in (self.lib.roctxProfilerResume, self.lib.roctxProfilerPause):
                f.argtypes = [ctypes.c_uint64]
                f.restype = None

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "host_cores": os.cpu_count(),
            "cores_available": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(state, spec, budget_s=20.0, max_iter=50, max_dets=4_000_000):
    """The oracle, single thread, continuing from a bounded sample of the GPU's
    state at the start of the timed window: every k-th determinant of the list
    in key order (at most max_dets), with the same shift and iteration, for as
    many whole iterations as fit in about budget_s seconds (at least one). Work
    per walker update is what is compared; the sample keeps the oracle's run
    short."""
    from oracle import oracle as O
    keys_all, pops_all, e, (sh, nprev, vary) = state
    k = max(1, -(-len(pops_all) // max_dets))
    keys, pops = keys_all[::k], pops_all[::k]
    s, q = spec["system"], spec["qmc"]
    sysd = O.System.ueg(s["rs"], s["ecut_n2"], s["n_alpha"], s["n_beta"])
    run = O.Run(sysd, O.make_qmc(tau=q["tau"], seed=q["rng_seed"], init_pop=q["init_pop"],
                                 target_population=q["target_population"], shift_period=q["shift_period"],
                                 shift_damping=q["shift_damping"], excit_gen=O.EXGEN_UEG,
                                 initiator=q.get("initiator", 1), initiator_threshold=q["initiator_threshold"],
                                 fixed_point_bits=q["fixed_point_bits"], spawn_cutoff=q["spawn_cutoff"],
                                 method=q.get("method", 0), ccmc_truncation=q.get("ccmc_truncation", 0)))
    run.import_walkers(keys, pops, shift=sh, iteration=int(e["iteration"]), vary=vary, n_prev=max(1, nprev // k))
    scale = 2.0 ** q["fixed_point_bits"]
    nw_prev = run.estimators()["n_walkers_units"]
    upd, it = 0.0, 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0 < budget_s or it == 0) and it < max_iter:
        run.step(1)
        upd += nw_prev / scale
        nw_prev = run.estimators()["n_walkers_units"]
        it += 1
        print(f"# oracle iteration {it}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    out = {"value": upd / dt, "unit": "walker updates/s", "cores": 1, "kind": "oracle",
           "sample": (f"{it} iterations ({e['iteration'] + 1}..{e['iteration'] + it}) from every {k}-th "
                      f"determinant of the GPU list at the start of the timed window ({len(pops)} of "
                      f"{len(pops_all)} determinants, {abs(pops.astype('int64')).sum() / scale:.4g} walkers), "
                      f"single thread") if k > 1 else
                     (f"{it} iterations ({e['iteration'] + 1}..{e['iteration'] + it}) from the whole GPU list at "
                      f"the start of the timed window ({len(pops)} entries, "
                      f"{abs(pops.astype('int64')).sum() / scale:.4g} walkers), single thread")}
    out.update(host_cpu())
    return out


def batch_capacity(inst):
    """Determinant and spawn capacities for a group of instances. Death and
    cloning shrink populations continuously, so an instance can hold tens of
    determinants per walker (up to about 30 measured at 123 plane waves): the
    main list gets 40 entries per target walker, the spawn list 4 spawns."""
    def cap(members, n_now=0):
        tot = sum(inst[i][1]["target_population"] for i in members)
        return int(max(40 * tot, 2 * n_now)), int(4 * tot)
    return cap


HIST_FIELDS = ("iteration", "n_walkers_units", "n_occupied", "ref_pop_units", "n_spawned", "n_spawn_events",
               "death_sum", "spawn_sum", "rejected_sum", "n_rejected_units", "n_sign_flips", "num_limbs", "shift")


def run_batch64(args):
    """64 independent electron-gas instances batched (one context per key width,
    graph replay, autotuned launch geometry) against the same 64 instances run
    one after another by the plain path: same keys, same iterations, timed over
    the same window. Batched instance i and plain run i are the same
    computation, so their estimator histories over the window must agree
    exactly; the count of instances that do is reported."""
    import torch
    from paper_1811_11679_amd import autotune
    from paper_1811_11679_amd import batch as B
    from paper_1811_11679_amd import fciqmc as F
    from paper_1811_11679_amd import workloads

    inst = workloads.batch64()
    n = len(inst)
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    cap = batch_capacity(inst)
    bt = B.Batch(inst, capacity=cap)
    log(f"batch: {n} instances in {len(bt.contexts)} contexts "
        f"(key words {[c.W for c in bt.contexts]}, instances {[len(g) for g in bt.groups]})")
    t_w0 = time.perf_counter()

    def warm_to(target):
        done = int(bt.estimators(0)["iteration"])
        while done < target:
            k = min(250, target - done)
            bt.step(k)
            done += k
            tot = sum(bt.estimators(i)["n_walkers_units"] for i in range(n)) / 256.0
            log(f"batch warmup {done}: total N_w {tot:.4g}, {time.perf_counter() - t_w0:.1f} s")

    # launch geometry is searched near the end of the equilibration, where the
    # populations are close to their targets, one context at a time; it does
    # not change the results
    # the workload runs 5000 iterations and times the last 1000: 4000 of
    # equilibration, then --warmup more
    equil = 4000 + args.warmup
    warm_to(int(equil * 0.8))
    tuned = [autotune.tune(c, iters=3, log=lambda m, k=k: log(f"context {k}: {m}"))
             for k, c in enumerate(bt.contexts)]
    warm_to(equil)
    t_start = int(bt.estimators(0)["iteration"])
    e_start = [bt.estimators(i) for i in range(n)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(args.steps)
    bt.synchronize()
    dt_b = time.perf_counter() - t0
    hist_b = [bt.history(i) for i in range(n)]
    upd_b = sum((e_start[i]["n_walkers_units"] + sum(x["n_walkers_units"] for x in hist_b[i][:-1])) / 256.0
                for i in range(n))
    groups = [len(g) for g in bt.groups]
    bt.close()
    torch.cuda.empty_cache()
    log(f"batched: iterations {t_start + 1}..{t_start + args.steps} in {dt_b:.2f} s, "
        f"{upd_b / dt_b:.4g} walker updates/s")
    # plain path, one instance after another from the same initial state with
    # the same keys; only the same window of iterations is timed
    upd_p, dt_p, same = 0.0, 0.0, 0
    for i, (sysd, q) in enumerate(inst):
        mc, sc = cap([i])
        ctx = F.Context([F.make_system(F.UEG, **{k: v for k, v in sysd.items() if k != "kind"})],
                        [F.make_qmc(excit_gen=F.UEG, **q)], main_capacity=mc, spawn_capacity=sc, graph=True)
        ctx.step(t_start)
        e0 = ctx.estimators()
        ctx.stream.synchronize()
        t0 = time.perf_counter()
        ctx.step(args.steps)
        ctx.stream.synchronize()
        dt = time.perf_counter() - t0
        h = ctx.history()
        ctx.close()
        u = (e0["n_walkers_units"] + sum(x["n_walkers_units"] for x in h[:-1])) / 256.0
        ok = len(h) == len(hist_b[i]) and all(a[f] == b[f] for a, b in zip(h, hist_b[i]) for f in HIST_FIELDS)
        same += int(ok)
        upd_p += u
        dt_p += dt
        log(f"plain instance {i}: {u / dt:.4g} walker updates/s over the window ({dt:.2f} s), "
            f"{'identical to' if ok else 'DIFFERENT from'} the batched instance")
    out = {
        "metric": METRIC,
        "value": upd_b / dt_b,
        "unit": "walker updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_b * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batch64_ueg14_rs{0.5,1,2,4}_pw{19,27,57,123}_targets1e5-2e6",
                   "instances": n, "contexts": len(groups), "instances_per_context": groups,
                   "timed_iterations": f"{t_start + 1}..{t_start + args.steps}", "graph_replay": True,
                   "autotuned_blocks": tuned, "parallelism": "single GPU"},
        "plain_sequential": {"value": upd_p / dt_p, "unit": "walker updates/s", "seconds": dt_p,
                             "instances_identical_to_batched": same},
        "batched_over_plain": (upd_b / dt_b) / (upd_p / dt_p),
        "walker_updates": upd_b,
    }
    print(json.dumps(out))


def run_mol30(args):
    """Semi-stochastic FCIQMC on the seeded molecular-like Hamiltonian (30
    orbitals, 8 + 8 electrons, heat-bath doubles): D = 2000 most highly
    weighted determinants (one space shared by the replicas when there are
    several), total target 1e7 walkers split evenly over the replicas, the
    projection in FP64 and in split BF16 x3 / FP32 on MFMA, each run from the
    same start with the same keys."""
    from paper_1811_11679_amd import fciqmc as F
    from paper_1811_11679_amd import synth, workloads

    R = args.replicas
    w = workloads.MOL30
    h1, eri = synth.molecular_integrals()
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    # equilibration of 4000 iterations (part of the workload) plus --warmup;
    # the deterministic space is chosen 300 iterations before the timed window
    equil = 4000 + args.warmup
    start = max(equil - 300, 1)
    tgt = 1e7 / R
    results = {}
    for prec in (F.SS_FP64, F.SS_SPLIT_BF16):
        name = "fp64" if prec == F.SS_FP64 else "split_bf16x3"
        sysd = F.make_system(F.MOLECULAR, n_orb=30, n_alpha=8, n_beta=8, h1=h1, eri=eri)
        qs = [F.make_qmc(excit_gen=F.MOLECULAR, **dict(w["qmc"], target_population=tgt, init_pop=tgt / 20,
                                                       replica_id=r)) for r in range(R)]
        ss = F.SemiStoch(size=2000, start_iteration=start, precision=prec, check_period=10, shared=1 if R > 1 else 0)
        ctx = F.Context([sysd] * R, qs, ss, main_capacity=args.main_capacity, spawn_capacity=args.spawn_capacity,
                        graph=True)
        t0 = time.perf_counter()
        done = 0
        while done < equil:
            k = min(250, equil - done)
            ctx.step(k)
            done += k
            nw = sum(ctx.estimators(r)["n_walkers_units"] for r in range(R)) / 256.0
            log(f"{name} warmup {done}: N_w {nw:.4g}, {time.perf_counter() - t0:.1f} s")
        e0 = [ctx.estimators(r) for r in range(R)]
        # timed window under graph replay, then a kernel window of at most 200
        # iterations with an event around every launch
        ctx.stream.synchronize()
        t1 = time.perf_counter()
        ctx.step(args.steps)
        ctx.stream.synchronize()
        dt = time.perf_counter() - t1
        hists = [ctx.history(r) for r in range(R)]
        ctx.set_timing(True)
        ctx.step(min(args.steps, 200))
        ctx.stream.synchronize()
        kt, niter = ctx.kernel_times()
        it_ms = sorted(ctx.iteration_times())
        ctx.set_timing(False)
        upd = sum((e0[r]["n_walkers_units"] + sum(h["n_walkers_units"] for h in hists[r][:-1])) / 256.0
                  for r in range(R))
        errs = [h["ss_error"] for hh in hists for h in hh if h["ss_error"] > 0]
        num = sum(h["proj_numerator"] for hh in hists for h in hh)
        den = sum(h["ref_pop_units"] for hh in hists for h in hh) / 256.0
        results[name] = {
            "walker_updates_per_s": upd / dt,
            "ms_per_iteration": dt * 1e3 / args.steps,
            "iteration_ms_device_median": it_ms[len(it_ms) // 2],
            "projection_ms_per_iteration": kt["det_project"] / max(niter, 1),
            "gather_ms_per_iteration": kt["det_gather"] / max(niter, 1),
            "fp64_check_ms_per_iteration": kt["det_check"] / max(niter, 1),
            "kernel_ms_per_iteration": {k: v / max(niter, 1) for k, v in kt.items()
                                        if v / max(niter, 1) > 0.005 and not k.startswith("ccmc")},
            "projected_energy_window": num / den if den else None,
            "ss_error_max": max(errs) if errs else None,
            "ss_error_bound": hists[0][-1]["ss_error_bound"],
            "walkers_end": sum(hh[-1]["n_walkers_units"] for hh in hists) / 256.0,
            "determinants_end": sum(hh[-1]["n_occupied"] for hh in hists),
        }
        log(f"{name}: {results[name]['walker_updates_per_s']:.4g} walker updates/s, projection "
            f"{results[name]['projection_ms_per_iteration']:.4f} ms/iteration")
        ctx.close()
    split, fp = results["split_bf16x3"], results["fp64"]
    out = {
        "metric": METRIC,
        "value": split["walker_updates_per_s"],
        "unit": "walker updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": split["ms_per_iteration"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (projection bf16x3/fp32 on MFMA)",
        "data": "synthetic",
        "config": {"workload": f"mol30_semistochastic_D2000_R{R}_target1e7", "replicas": R,
                   "deterministic_space": 2000, "shared_space": R > 1, "selection_iteration": start,
                   "timed_iterations": f"{equil + 1}..{equil + args.steps}", "graph_replay": True,
                   "kernel_timing_iterations": f"{equil + args.steps + 1}..{equil + args.steps + min(args.steps, 200)}",
                   "parallelism": "single GPU"},
        "fp64": fp,
        "split_bf16x3": split,
        "split_over_fp64_walker_updates": split["walker_updates_per_s"] / fp["walker_updates_per_s"],
        "split_over_fp64_projection_speed": fp["projection_ms_per_iteration"] / split["projection_ms_per_iteration"],
    }
    print(json.dumps(out))


def single_spec(args):
    """The single-instance workloads: 14-electron gas (default), the
    54-electron gas with its split-precision deterministic space, and coupled
    cluster Monte Carlo at CCSD on the 14-electron gas."""
    from paper_1811_11679_amd import fciqmc as F
    from paper_1811_11679_amd import workloads
    if args.workload == "ccmc":
        w = workloads.UEG14_CCSD
        return dict(name="ccmc", w=w, system=w["system"], qmc=dict(w["qmc"]), ss=None,
                    equilibration=w["equilibration"],
                    config={"workload": "ccmc_ccsd_ueg14_rs1_57pw", "method": "CCMC", "truncation": "CCSD",
                            "electrons": 14, "rs": 1.0, "plane_waves": 57, "fixed_point": "1/256"})
    if args.workload == "ueg14":
        w = workloads.UEG14
        return dict(name="ueg14", w=w, system=w["system"], qmc=dict(w["qmc"]), ss=None,
                    equilibration=w["equilibration"],
                    config={"workload": "ueg14_rs1_57pw_initiator_target1e7", "electrons": 14, "rs": 1.0,
                            "plane_waves": 57, "fixed_point": "1/256", "initiator_threshold": 3.0})
    w = workloads.UEG54
    q = dict(w["qmc"])
    for k, a in (("target_population", "target"), ("init_pop", "init_pop"), ("initial_shift", "initial_shift"),
                 ("shift_damping", "shift_damping"), ("tau", "tau")):
        if getattr(args, a) is not None:
            q[k] = getattr(args, a)
    equil = w["equilibration"]
    ss = F.SemiStoch(size=w["semistoch"]["size"], start_iteration=w["semistoch"]["start_iteration"],
                     precision=F.SS_SPLIT_BF16, check_period=10)
    return dict(name="ueg54", w=w, system=w["system"], qmc=q, ss=ss, equilibration=equil,
                config={"workload": "ueg54_rs1_251pw_initiator_D8192_split", "electrons": 54, "rs": 1.0,
                        "plane_waves": 251, "fixed_point": "1/256", "initiator_threshold": 3.0,
                        "deterministic_space": w["semistoch"]["size"], "projection": "bf16x3/fp32 MFMA"})


def run_single(args):
    """One instance: equilibrate (part of the workload), --warmup more
    iterations, then --steps timed iterations under graph replay, then as many
    again with per-kernel events for the roofline."""
    import torch
    from paper_1811_11679_amd import fciqmc as F

    spec = single_spec(args)
    s, q = spec["system"], spec["qmc"]
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    sysd = F.make_system(F.UEG, rs=s["rs"], ecut_n2=s["ecut_n2"], n_alpha=s["n_alpha"], n_beta=s["n_beta"])
    ctx = F.Context([sysd], [F.make_qmc(excit_gen=F.UEG, **q)], spec["ss"], main_capacity=args.main_capacity,
                    spawn_capacity=args.spawn_capacity, graph=True)
    log(f"workspace {ctx.workspace.numel() / 1e9:.1f} GB, key words {ctx.W}")
    scale = 2.0 ** q["fixed_point_bits"]
    t_w0 = time.perf_counter()
    pre = spec["equilibration"] + args.warmup
    # tile shapes and block counts are searched on the live run once the
    # population is at its working size (results do not depend on them)
    tune_at = pre // 2 if not args.no_autotune else None
    tuned = None
    done = 0
    while done < pre:
        k = min(250, pre - done)
        if tune_at is not None and done < tune_at < done + k:
            k = tune_at - done
        ctx.step(k)
        done += k
        e = ctx.estimators()
        log(f"equilibration {done}/{pre}: N_w {e['n_walkers_units'] / scale:.4g} walkers, "
            f"{e['n_occupied']} determinants, N_0 {e['ref_pop_units'] / scale:.4g}, shift {e['shift']:.5f}, "
            f"E_proj {e['proj_energy']:.5f}, {time.perf_counter() - t_w0:.1f} s")
        if tune_at is not None and done == tune_at:
            from paper_1811_11679_amd import autotune
            tuned = autotune.tune(ctx, iters=3, log=log)
            done = int(ctx.estimators()["iteration"])
    warm_s = time.perf_counter() - t_w0
    e_start = ctx.estimators()
    start_state = None
    if not args.no_cpu_baseline:
        keys, pops = ctx.export()
        start_state = (keys, pops, e_start, ctx.shift_state())
    prof = ProfilerRegion()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    prof.resume()
    t0 = time.perf_counter()
    ev0.record(ctx.stream)
    ctx.step(args.steps)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hist = ctx.history()[-args.steps:]
    prev = [e_start] + hist[:-1]
    upd = sum(h["n_walkers_units"] for h in prev) / scale
    dev_ms = ev0.elapsed_time(ev1)
    # kernel window: same length (at most 200 iterations), an event around every launch
    nk = min(args.steps, 200)
    e_k0 = ctx.estimators()
    ctx.set_timing(True)
    ctx.step(nk)
    torch.cuda.synchronize()
    prof.pause()
    ctx.set_timing(False)
    hk = ctx.history()[-nk:]
    prevk = [e_k0] + hk[:-1]
    ktimes, niter = ctx.kernel_times()
    stages = ctx.stage_times()
    it_ms = sorted(ctx.iteration_times())
    dets = sum(h["n_occupied"] for h in prev)
    spawned = sum(h["n_spawned"] for h in hist)
    ds_active = spec["ss"] is not None
    is_cc = q.get("method", 0) == F.CCMC
    cc = (q["ccmc_truncation"], s["n_alpha"] + s["n_beta"], q["fixed_point_bits"]) if is_cc else None
    tot_bytes = {}
    for a, b in zip(prevk, hk):
        for k, v in algorithmic_bytes(a, b, ctx.W, ds_active=ds_active, ccmc=cc).items():
            tot_bytes[k] = tot_bytes.get(k, 0) + v
    cand = {"spawn": ["spawn"], "merge": ["merge"], "reduce": ["reduce"], "new_diag": ["new_diag"],
            "sort_pass": [f"sort_pass{p}" for p in range(8)]}
    if is_cc:
        # the cluster slot holds the prefix scan and the cluster sampler (two launches)
        cand["ccmc_clusters"] = ["ccmc_clusters"]
    best = max(cand, key=lambda g: sum(ktimes[k] for k in cand[g]))
    launches = niter * len(cand[best])
    avg_ms = sum(ktimes[k] for k in cand[best]) / max(launches, 1)
    bytes_per_launch = sum(tot_bytes[k] for k in cand[best]) / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    ann_ms = stages["sort"] + stages["reduce"] + stages["merge"]
    ann_bytes = sum(tot_bytes[k] for k in tot_bytes if k.startswith("sort") or k in ("reduce", "merge"))
    hwin = hist + hk
    errs = [h["ss_error"] for h in hwin if h.get("ss_error", 0) > 0]
    cfg = dict(spec["config"])
    cfg.update({"key_words": ctx.W, "tau": q["tau"], "target_walkers": q["target_population"],
                "init_pop": q["init_pop"], "shift_damping": q["shift_damping"],
                "equilibration_iterations": spec["equilibration"],
                "timed_iterations": f"{e_start['iteration'] + 1}..{hist[-1]['iteration']}",
                "kernel_timing_iterations": f"{e_k0['iteration'] + 1}..{hk[-1]['iteration']}",
                "graph_replay": True, "autotuned": tuned, "tiles": ctx.get_tiles(), "blocks": ctx.get_launch(),
                "parallelism": "single GPU"})
    out = {
        "metric": METRIC,
        "value": upd / dt,
        "unit": "walker updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if spec["ss"] is None else "f64 (deterministic projection bf16x3/fp32 on MFMA)",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "kernel": best, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(best, spec["name"]),
                     "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch},
        "device_ms_per_step": dev_ms / args.steps,
        "annihilation_gbps_algorithmic": ann_bytes / (ann_ms * 1e-3) / 1e9 if ann_ms > 0 else None,
        "iteration_ms_device_kernel_window": {"median": it_ms[len(it_ms) // 2], "p90": it_ms[(9 * len(it_ms)) // 10],
                                              "min": it_ms[0], "max": it_ms[-1]} if it_ms else None,
        "determinant_updates_per_s": dets / dt,
        "spawns_per_s": spawned / dt,
        "stage_ms_per_iteration": {k: v / max(niter, 1) for k, v in stages.items()},
        # (the two CCMC slots time only the gap between two events on the FCIQMC path)
        "kernel_ms_per_iteration": {k: v / max(niter, 1) for k, v in ktimes.items()
                                    if v > 0 and (is_cc or not k.startswith("ccmc"))},
        "walkers_start": e_start["n_walkers_units"] / scale,
        "walkers_end": hist[-1]["n_walkers_units"] / scale,
        "determinants_start": e_start["n_occupied"],
        "determinants_end": hist[-1]["n_occupied"],
        "spawned_per_iteration": spawned / len(hist),
        "ref_pop_start": e_start["ref_pop_units"] / scale,
        "ref_pop_end": hist[-1]["ref_pop_units"] / scale,
        "shift_mean_window": sum(h["shift"] for h in hist) / len(hist),
        "proj_energy_window": (sum(h["proj_numerator"] for h in hist) / sum(h["ref_pop_units"] for h in hist) * scale)
        if sum(h["ref_pop_units"] for h in hist) else None,
        "warmup_s": warm_s,
    }
    if ds_active:
        out["ss_error_max"] = max(errs) if errs else None
        out["ss_error_bound"] = hwin[-1]["ss_error_bound"]
        out["projection_ms_per_iteration"] = ktimes["det_project"] / max(niter, 1)
    ctx.close()
    if args.calibrate_copy:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE per
        # dispatch scale the counters of the FCIQMC kernels to bytes
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        prof.resume()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        prof.pause()
        out["copy_calibration_bytes"] = 1 << 30
    if start_state is not None:
        out["cpu_baseline"] = cpu_baseline(start_state, spec)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed iterations")
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed iterations after the workload's own equilibration (never shortens it)")
    ap.add_argument("--main-capacity", type=int, default=None,
                    help="determinant capacity (default 2^28; ueg54: 3.3e8)")
    ap.add_argument("--spawn-capacity", type=int, default=None, help="spawn capacity (default 2^27; ueg54: 2e8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shapes and block counts (no search during equilibration)")
    ap.add_argument("--target", type=float, default=None, help="ueg54: target walkers")
    ap.add_argument("--init-pop", type=float, default=None, help="ueg54: initial walkers on the reference")
    ap.add_argument("--shift-damping", type=float, default=None, help="ueg54: shift damping (zeta)")
    ap.add_argument("--initial-shift", type=float, default=None, help="ueg54: initial shift (Hartree, relative to H_00)")
    ap.add_argument("--tau", type=float, default=None, help="ueg54: time step")
    ap.add_argument("--workload", default="ueg14", choices=["ueg14", "batch64", "mol30", "ueg54", "ccmc"],
                    help="ueg14: the plain single-instance path; ueg54: the large single instance; batch64: 64 "
                         "batched instances vs plain runs; mol30: semi-stochastic molecular runs, FP64 vs split; "
                         "ccmc: coupled cluster Monte Carlo at CCSD on the 14-electron gas")
    ap.add_argument("--replicas", type=int, default=1, help="mol30: replicas sharing one deterministic space")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of 1 GiB (4 times) for counter calibration")
    args = ap.parse_args()
    big = args.workload == "ueg54"
    cc = args.workload == "ccmc"  # about 1.8e3 amplitudes, up to ~3e7 spawn records per iteration
    if args.main_capacity is None:
        args.main_capacity = 330_000_000 if big else (1 << 20 if cc else 1 << 28)
    if args.spawn_capacity is None:
        args.spawn_capacity = 200_000_000 if big else (1 << 26 if cc else 1 << 27)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding across GPUs is "
              "designed but not implemented", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("--steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return run_batch64(args)
    if args.workload == "mol30":
        return run_mol30(args)
    return run_single(args)


if __name__ == "__main__":
    main()
