"""Post-hoc blocking analysis of correlated series (test infrastructure only).

The plain definition that the library's on-the-fly accumulator must
reproduce (Sec. 3.1: the reblocking analysis of Flyvbjerg and Petersen).
Level 0 is the series itself; level k + 1 averages consecutive pairs of
level-k values, dropping an unpaired last value; at every level the block
values give a mean and a sample covariance (numpy, two-pass). The optimal
level is the first whose block length B = 2^k satisfies
B^3 > 2 n (e_k / e_0)^4 (Lee, Needs and Towler, Phys. Rev. E 83, 066706);
the ratio of two means carries its first-order (delta-method) error.

Only the tests import this module.
"""
from __future__ import annotations

import numpy as np


def block_levels(x):
    """x: (n, S) observations. Returns [(n_blocks, mean[S], cov[S, S])] for
    every level with at least two block values."""
    cur = np.asarray(x, dtype=np.float64)
    if cur.ndim == 1:
        cur = cur[:, None]
    out = []
    while len(cur) >= 2:
        n = len(cur)
        mean = cur.mean(axis=0)
        dev = cur - mean
        cov = dev.T @ dev / (n - 1)
        out.append((n, mean, cov))
        m = n // 2
        cur = (cur[0:2 * m:2] + cur[1:2 * m:2]) * 0.5
    return out


def std_error(levels, k, s):
    n, _, cov = levels[k]
    return float(np.sqrt(cov[s, s] / n))


def optimal_level(levels, s):
    n0 = levels[0][0]
    e0 = std_error(levels, 0, s)
    if e0 == 0.0:
        return 0
    for k in range(len(levels)):
        if 2.0 ** (3 * k) > 2.0 * n0 * (std_error(levels, k, s) / e0) ** 4:
            return k
    return -1


def ratio(levels, k, a, b):
    """mean_a / mean_b at level k and its first-order standard error."""
    n, mean, cov = levels[k]
    q = mean[a] / mean[b]
    var = (cov[a, a] - 2.0 * q * cov[a, b] + q * q * cov[b, b]) / n / mean[b] ** 2
    return float(q), float(np.sqrt(max(var, 0.0)))
