"""On-the-fly reblocking: the post-hoc oracle pinned to closed forms, then
the library's accumulator (host code, no GPU) against the oracle."""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle import reblock as R


def _ar1(n, phi, rng):
    """x_t = phi x_{t-1} + e_t, unit normal innovations, stationary start."""
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1.0 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


# ---- pins of the oracle ----------------------------------------------------

def test_block_values_are_means_of_consecutive_blocks():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1000, 2))
    lv = R.block_levels(x)
    for k in range(1, 6):
        b = 2 ** k
        nb = len(x) // b
        direct = x[: nb * b].reshape(nb, b, 2).mean(axis=1)
        assert lv[k][0] == nb
        np.testing.assert_allclose(lv[k][1], direct.mean(axis=0), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(lv[k][2], np.cov(direct, rowvar=False, ddof=1), rtol=1e-9, atol=1e-15)


def test_iid_error_is_sigma_over_root_n_at_every_level():
    rng = np.random.default_rng(2)
    n = 1 << 16
    lv = R.block_levels(2.0 * rng.standard_normal(n))
    exact = 2.0 / math.sqrt(n)
    for k in range(0, 8):
        nb = lv[k][0]
        # relative error of a standard-error estimate from nb blocks ~ 1/sqrt(2 nb)
        assert abs(R.std_error(lv, k, 0) / exact - 1.0) < 5.0 / math.sqrt(2 * nb), k
    # uncorrelated data: e_k / e_0 ~ 1, so the criterion asks for B^3 > 2 n, B = 64 at n = 2^16
    assert R.optimal_level(lv, 0) in (5, 6, 7)


def test_ar1_error_matches_the_closed_form_at_the_optimal_level():
    # variance of the mean of a stationary AR(1) series: (1 + phi) / ((1 - phi) (1 - phi^2) n)
    rng = np.random.default_rng(3)
    n, phi = 1 << 18, 0.9
    lv = R.block_levels(_ar1(n, phi, rng))
    exact = math.sqrt((1 + phi) / ((1 - phi) * (1 - phi * phi) * n))
    k = R.optimal_level(lv, 0)
    assert 3 <= k <= 12
    assert abs(R.std_error(lv, k, 0) / exact - 1.0) < 0.12
    # level 0 ignores the correlation: it underestimates by sqrt((1 - phi) / (1 + phi))
    assert R.std_error(lv, 0, 0) / exact < 0.3


def test_ratio_error_matches_the_spread_of_independent_runs():
    # correlated numerator and denominator: the covariance term matters
    rng = np.random.default_rng(4)
    ratios, errs = [], []
    for _ in range(300):
        b = 5.0 + rng.standard_normal(512)
        a = 2.0 * b + 0.5 * rng.standard_normal(512) + 1.0
        lv = R.block_levels(np.stack([a, b], axis=1))
        q, e = R.ratio(lv, 0, 0, 1)
        ratios.append(q)
        errs.append(e)
    spread = float(np.std(ratios, ddof=1))
    assert abs(float(np.mean(errs)) / spread - 1.0) < 0.15
    # dropping the covariance term would overestimate by a factor > 3 here
    lv = R.block_levels(np.stack([a, b], axis=1))
    n, mean, cov = lv[0]
    no_cov = math.sqrt((cov[0, 0] + (mean[0] / mean[1]) ** 2 * cov[1, 1]) / n) / mean[1]
    assert no_cov > 3 * R.ratio(lv, 0, 0, 1)[1]


# ---- the library's accumulator against the oracle --------------------------

def _lib():
    from paper_1811_11679_amd import fciqmc as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    return F


def test_on_the_fly_levels_equal_the_post_hoc_analysis():
    _lib()
    from paper_1811_11679_amd import reblock as RB
    rng = np.random.default_rng(5)
    n = 5000  # not a power of two: incomplete last blocks at many levels
    x = np.stack([_ar1(n, 0.8, rng) + 3.0, 100.0 + 10.0 * _ar1(n, 0.95, rng), rng.standard_normal(n)], axis=1)
    acc = RB.OnTheFly(3, n_levels=20)
    for row in x:
        acc.add(row)
    post = R.block_levels(x)
    got = acc.levels()
    assert len(got) == len(post)
    for k, ((na, ma, ca), (nb, mb, cb)) in enumerate(zip(got, post)):
        assert na == nb, k
        np.testing.assert_allclose(ma, mb, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(ca, cb, rtol=1e-9, atol=1e-12)
    for s in range(3):
        assert acc.optimal(s) == R.optimal_level(post, s)
    for k in range(len(post)):
        q1, e1 = acc.ratio(k, 1, 0)
        q2, e2 = R.ratio(post, k, 1, 0)
        assert q1 == pytest.approx(q2, rel=1e-12)
        assert e1 == pytest.approx(e2, rel=1e-8)
    acc.close()


def test_on_the_fly_edge_cases_and_argument_checks():
    F = _lib()
    from paper_1811_11679_amd import reblock as RB
    L = F.load_library()
    h = ctypes.c_void_p()
    assert L.fq_reblock_create(ctypes.byref(h), 0, 10) == F.FQ_EINVAL
    assert L.fq_reblock_create(ctypes.byref(h), 3, 0) == F.FQ_EINVAL
    assert L.fq_reblock_create(None, 3, 10) == F.FQ_EINVAL
    acc = RB.OnTheFly(2, n_levels=4)
    assert acc.optimal(0) == -1  # no data yet
    acc.add([1.0, 2.0])
    n, m, c = acc.level(0)
    assert n == 1 and np.all(np.isnan(c))
    with pytest.raises(F.FqError):
        acc.add([float("nan"), 1.0])
    assert acc.level(0)[0] == 1  # the rejected observation left no trace
    for _ in range(20):
        acc.add([1.0, 2.0])
    assert acc.optimal(0) == 0  # a constant series
    q, e = acc.ratio(0, 0, 1)
    assert q == 0.5 and e == 0.0
    with pytest.raises(F.FqError):
        acc.level(4)
    with pytest.raises(F.FqError):
        acc.optimal(2)
    acc.close()


class _FakeContext:
    """Stands in for a library context: replays a precomputed estimator series."""

    def __init__(self, rows):
        self.rows = rows
        self.t = 0
        self.last = []

    def step(self, k):
        self.last = [dict(iteration=self.t + 1 + i, shift=float(self.rows[self.t + i][0]),
                          proj_numerator=float(self.rows[self.t + i][1]), ref_pop_units=float(self.rows[self.t + i][2]))
                     for i in range(k)]
        self.t += k

    def history(self, instance=0):
        return self.last

    def estimators(self, instance=0):
        return {"iteration": self.t}


def test_run_until_error_stops_at_the_first_qualifying_check():
    _lib()
    from paper_1811_11679_amd import reblock as RB
    rng = np.random.default_rng(6)
    n = 1 << 15
    den = 100.0 + 5.0 * _ar1(n, 0.9, rng)
    num = -0.5 * den + 2.0 * _ar1(n, 0.9, rng)
    rows = np.stack([-0.5 + 0.1 * _ar1(n, 0.9, rng), num, den], axis=1)
    ctx = _FakeContext(rows)
    obs = []
    start, block, target, min_blocks = 200, 256, 0.004, 16
    res = RB.run_until_error(ctx, target, start, block=block, max_iterations=n, observations=obs, min_blocks=min_blocks)
    assert res["converged"]
    np.testing.assert_array_equal(np.array(obs), rows[start:res["iteration"]])

    def decide(x):
        lv = R.block_levels(x)
        k1, k2 = R.optimal_level(lv, 1), R.optimal_level(lv, 2)
        if min(k1, k2) < 0:
            return False, None
        k = max(k1, k2)
        e, err = R.ratio(lv, k, 1, 2)
        return lv[k][0] >= min_blocks and err <= target, (k, e, err)

    ok, (k, e, err) = decide(rows[start:res["iteration"]])
    assert ok and k == res["level"]
    assert res["proj_energy"] == pytest.approx(e, rel=1e-12) and res["proj_energy_error"] == pytest.approx(err, rel=1e-8)
    assert not decide(rows[start:res["iteration"] - block])[0]
    # an unreachable target runs to the limit and reports no convergence
    ctx2 = _FakeContext(rows)
    res2 = RB.run_until_error(ctx2, 1e-9, start, block=block, max_iterations=4096)
    assert ctx2.t == 4096 and (res2 is None or not res2["converged"])
