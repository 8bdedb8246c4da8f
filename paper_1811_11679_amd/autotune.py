"""Tile-shape and launch-geometry search for the persistent kernels of one
context.

Every persistent kernel takes its tiles by atomic ticket (or by grid stride),
and the look-back chains are ordered by ticket, so the walker lists and
estimators depend neither on the tile shapes (the compiled variants of
spawning attempts, merge positions and radix-sort keys per thread) nor on how
many blocks are launched: only the speed does. The search therefore runs on
the live simulation (during its equilibration) and costs no extra work: each
candidate is timed over a few iterations with per-kernel events, normalised by
the work those iterations carried, and the fastest is kept. Tile shapes are
chosen first (they change how many blocks fit a compute unit), then block
counts, one kernel at a time.
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
# the kernel (work measure) and event slots of each tile-shape knob
_TILE_KERNEL = {"spawn_items": "spawn", "merge_items": "merge", "sort_items": "sort"}
_TILE_SLOTS = {"spawn_items": ["spawn_partition", "spawn"], "merge_items": ["merge_partition", "merge"],
               "sort_items": [f"sort_pass{p}" for p in range(8)]}


def candidates(n_cu, current):
    """Block counts tried for one kernel: multiples of the compute-unit count."""
    c = {n_cu * f for f in (1, 2, 3, 4, 6, 8, 12, 16)}
    c.add(int(current))
    return sorted(c)


def _trial(ctx, iters, kernel, slots=None):
    """Summed event time of the kernel's launches (or of the given event slots)
    over iters iterations, and the work they carried summed over every instance
    of the context."""
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
    return sum(kt[s] for s in (slots or _SLOTS[kernel])), max(work, 1)


def tune_tiles(ctx, iters=3, knobs=None, log=None):
    """Search the compiled tile-shape variants (F.TILE_VARIANTS) on the running
    context, advancing it by iters x (number of variants) iterations per knob.
    Returns {knob: value}; the context keeps the chosen shapes."""
    knobs = list(knobs or F.TILE_KNOBS)
    best = ctx.get_tiles()
    for k in knobs:
        scores = {}
        for v in F.TILE_VARIANTS[k]:
            ctx.set_tiles({k: v})
            ms, work = _trial(ctx, iters, _TILE_KERNEL[k], _TILE_SLOTS[k])
            scores[v] = ms / work
        choice = min(scores, key=scores.get)
        ctx.set_tiles({k: choice})
        best[k] = choice
        if log:
            log(f"autotune {k}: {choice} ({', '.join(f'{v}: {x * 1e9:.3g}' for v, x in sorted(scores.items()))} "
                f"ps per work unit)")
    return best


def tune(ctx, iters=3, kernels=None, n_cu=None, log=None, tiles=True):
    """Search tile shapes (unless tiles is False), then block counts for
    `kernels` (default: all tunable ones) on the running context, advancing it
    by iters x (number of candidates) iterations. Returns {kernel: blocks} and,
    under "tiles", the chosen shapes; the context keeps the choice."""
    if n_cu is None:
        n_cu = ctx.n_cu
    shapes = tune_tiles(ctx, iters, log=log) if tiles else ctx.get_tiles()
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
    best["tiles"] = shapes
    return best
