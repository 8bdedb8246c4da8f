"""Launch-geometry search for the persistent kernels of one context.

Every persistent kernel takes its tiles by atomic ticket (or by grid stride),
and the look-back chains are ordered by ticket, so the walker lists and
estimators do not depend on how many blocks are launched: only the speed does.
The search therefore runs on the live simulation (during its equilibration)
and costs no extra work: each candidate block count is timed over a few
iterations with per-kernel events, normalised by the work those iterations
carried, and the fastest is kept. Kernels are tuned one at a time, in the
order of their share of the iteration.
"""
from __future__ import annotations

from . import fciqmc as F

# which per-iteration quantity each kernel's time scales with
_WORK = {
    "spawn": lambda a, b: a["n_walkers_units"] + 64 * b["n_spawned"],
    "merge": lambda a, b: a["n_occupied"] + b["n_occupied"] + b["n_spawn_events"],
    "sort": lambda a, b: b["n_spawned"],
    "reduce": lambda a, b: b["n_spawned"],
    "new_diag": lambda a, b: b["n_occupied"],
}
_SLOTS = {
    "spawn": ["spawn"],
    "merge": ["merge"],
    "sort": [f"sort_pass{p}" for p in range(8)],
    "reduce": ["reduce", "reduce2"],
    "new_diag": ["new_diag"],
}


def candidates(n_cu, current):
    """Block counts tried for one kernel: multiples of the compute-unit count."""
    c = {n_cu * f for f in (1, 2, 3, 4, 6, 8, 12, 16)}
    c.add(int(current))
    return sorted(c)


def _trial(ctx, iters, kernel):
    """Summed event time of the kernel's launches over iters iterations, and the
    work they carried summed over every instance of the context."""
    e0 = [ctx.estimators(r) for r in range(ctx.R)]
    ctx.set_timing(True)
    try:
        ctx.step(iters)
        kt, _ = ctx.kernel_times()
    finally:
        ctx.set_timing(False)
    work = 0
    for r in range(ctx.R):
        hist = ctx.history(r)
        work += sum(_WORK[kernel](a, b) for a, b in zip([e0[r]] + hist[:-1], hist))
    return sum(kt[s] for s in _SLOTS[kernel]), max(work, 1)


def tune(ctx, iters=3, kernels=None, n_cu=None, log=None):
    """Search block counts for `kernels` (default: all tunable ones) on the
    running context, advancing it by iters x (number of candidates) iterations.
    Returns {kernel: blocks}; the context keeps the chosen geometry."""
    if n_cu is None:
        n_cu = ctx.n_cu
    kernels = list(kernels or F.LAUNCH_KERNELS)
    best = ctx.get_launch()
    report = {}
    for k in kernels:
        scores = {}
        for blocks in candidates(n_cu, best[k]):
            ctx.set_launch({k: blocks})
            ms, work = _trial(ctx, iters, k)
            scores[blocks] = ms / work
        choice = min(scores, key=scores.get)
        ctx.set_launch({k: choice})
        best[k] = choice
        report[k] = {b: s * 1e9 for b, s in scores.items()}  # ms per unit -> ps per unit
        if log:
            log(f"autotune {k}: {choice} blocks "
                f"({', '.join(f'{b}: {v:.3g}' for b, v in sorted(report[k].items()))} ps per work unit)")
    return best
