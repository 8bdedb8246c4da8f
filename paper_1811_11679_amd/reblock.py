"""On-the-fly blocking analysis and a run that stops at a requested error.

The accumulator lives in the C library (host code, no device call): every
iteration's estimators are added as they are produced, and the standard
errors of the shift and of the projected energy (numerator and reference
population averaged separately, then divided) are read at the blocking level
that Lee, Needs and Towler's criterion selects (Sec. 3.1 of the paper: the
reblocking analysis, done on the fly so that a calculation can end once its
error bar is small enough).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import fciqmc as F


class OnTheFly:
    """n_series series observed together, n_levels blocking levels."""

    def __init__(self, n_series, n_levels=40):
        self.lib = F.load_library()
        self.S = int(n_series)
        self.h = C.c_void_p()
        st = self.lib.fq_reblock_create(C.byref(self.h), self.S, int(n_levels))
        if st != F.FQ_OK:
            raise F.FqError(st, "fq_reblock_create: sizes out of range")
        self.L = int(n_levels)

    def add(self, x):
        a = np.ascontiguousarray(x, dtype=np.float64)
        if a.shape != (self.S,):
            raise ValueError(f"expected {self.S} values, got shape {a.shape}")
        st = self.lib.fq_reblock_add(self.h, a.ctypes.data_as(C.POINTER(C.c_double)))
        if st != F.FQ_OK:
            raise F.FqError(st, "fq_reblock_add: non-finite value")

    def level(self, k):
        """(n_blocks, means[S], covariance[S, S] of the block values)"""
        n = C.c_int64()
        mean = np.zeros(self.S)
        cov = np.zeros((self.S, self.S))
        st = self.lib.fq_reblock_level(self.h, int(k), C.byref(n), mean.ctypes.data_as(C.POINTER(C.c_double)),
                                       cov.ctypes.data_as(C.POINTER(C.c_double)))
        if st != F.FQ_OK:
            raise F.FqError(st, "fq_reblock_level: level out of range")
        return n.value, mean, cov

    def levels(self):
        """Every level with at least two blocks."""
        out = []
        for k in range(self.L):
            n, m, c = self.level(k)
            if n < 2:
                break
            out.append((n, m, c))
        return out

    def optimal(self, series):
        lv = C.c_int32()
        st = self.lib.fq_reblock_optimal(self.h, int(series), C.byref(lv))
        if st != F.FQ_OK:
            raise F.FqError(st, "fq_reblock_optimal: series out of range")
        return lv.value

    def ratio(self, k, num, den):
        r, e = C.c_double(), C.c_double()
        st = self.lib.fq_reblock_ratio(self.h, int(k), int(num), int(den), C.byref(r), C.byref(e))
        if st != F.FQ_OK:
            raise F.FqError(st, "fq_reblock_ratio: argument out of range")
        return r.value, e.value

    def close(self):
        if self.h:
            self.lib.fq_reblock_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SERIES = ("shift", "proj_numerator", "ref_pop_units")


def run_until_error(ctx, target_error, start_iteration, block=100, max_iterations=100_000, instance=0,
                    observations=None, min_blocks=16):
    """Advance ctx until the projected energy's standard error, at the
    blocking level the criterion selects for both its numerator and its
    denominator, is at most target_error (or max_iterations have run). An
    error read from fewer than min_blocks blocks is itself too uncertain to
    stop on (its relative error is about 1 / sqrt(2 (n_blocks - 1))), so the
    selected level must also hold at least min_blocks blocks.

    Iterations after start_iteration (equilibration excluded) are analysed.
    Returns a dict with the energy, its error, the shift and its error, the
    level used, the number of analysed iterations and whether the target was
    reached. If observations is a list, every analysed (shift, numerator,
    reference population) row is appended to it."""
    acc = OnTheFly(len(SERIES))
    done = 0
    result = None
    try:
        while done < max_iterations:
            k = min(block, max_iterations - done)
            ctx.step(k)
            done += k
            for h in ctx.history(instance):
                if h["iteration"] > start_iteration:
                    row = [float(h[s]) for s in SERIES]
                    acc.add(row)
                    if observations is not None:
                        observations.append(row)
            lv = [acc.optimal(i) for i in range(len(SERIES))]
            if min(lv[1], lv[2]) < 0:
                continue  # not enough data for the criterion yet
            kk = max(lv[1], lv[2])
            n, mean, cov = acc.level(kk)
            e, err = acc.ratio(kk, 1, 2)
            ks = lv[0]  # -1: the shift's error is not determined yet
            ns, ms, cs = acc.level(max(ks, 0))
            result = {"proj_energy": e, "proj_energy_error": err, "level": kk, "n_blocks": n,
                      "shift": ms[0], "shift_error": float(np.sqrt(cs[0, 0] / ns)) if ks >= 0 else float("nan"),
                      "shift_level": ks, "analysed_iterations": acc.level(0)[0],
                      "iteration": int(ctx.estimators(instance)["iteration"]),
                      "converged": n >= min_blocks and err <= target_error}
            if result["converged"]:
                break
        return result
    finally:
        acc.close()
