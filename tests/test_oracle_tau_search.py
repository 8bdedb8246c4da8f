"""The oracle's time-step search (the tutorial's tau_search), pinned.

* The running maximum of |H_ji| / p_gen that the search tracks equals the
  maximum over every outcome of the excitation generator from the reference
  (enumerated with forced random words), once one iteration has made enough
  attempts to draw every outcome.
* Over a run, tau never increases, changes only at shift updates, and after
  each change tau |H_ji| / p_gen <= 1 for the largest ratio seen.
* Without the search, tau is constant and no maximum is tracked.
"""
import math

import numpy as np

from oracle import oracle as O


def _word_for(index, n):
    """A random word that the multiply-shift choice maps to index of n."""
    return (index * (1 << 32) + n - 1) // n


def test_tracked_ratio_is_the_generator_maximum_from_the_reference():
    s = O.System.ueg(1.0, 2, 7, 7)  # 19 plane waves, one-word keys
    r = O.Run(s, O.make_qmc(tau=1e-5, seed=3, init_pop=2e5, target_population=1e9, excit_gen=O.EXGEN_UEG,
                            tau_search=1))
    keys, _ = r.export()
    d0 = keys[0]
    n_el, m = 14, 19
    npairs = n_el * (n_el - 1) // 2
    best = 0.0
    w1s = sorted({_word_for(a, m) for a in range(m)} | {_word_for(a, 2 * m) for a in range(2 * m)})
    for kp in range(npairs):
        w0 = _word_for(kp, npairs)
        for w1 in w1s:
            out = s.exgen(O.EXGEN_UEG, d0, [w0, w1, 0, 0])
            if out is None:
                continue
            _, pg, h = out
            if h != 0.0:
                best = max(best, abs(h) / pg)
    assert best > 0.0
    r.step(1)
    e = r.estimators()
    assert e["spawn_ratio_max"] == best
    # the first shift update (iteration 10) applies the bound
    r.step(9)
    e = r.estimators()
    assert e["tau"] <= 1.0 / best and e["tau"] <= 1e-5


def test_tau_never_increases_and_bounds_the_largest_spawn():
    s = O.System.hubbard()
    r = O.Run(s, O.make_qmc(tau=0.05, initial_shift=-4.0, tau_search=1))
    taus = []
    for it in range(1, 201):
        r.step(1)
        e = r.estimators()
        taus.append(e["tau"])
        if it % 10 != 0 and it > 1:
            assert taus[-1] == taus[-2], f"tau changed between shift updates (iteration {it})"
        if len(taus) > 1:
            assert taus[-1] <= taus[-2]
        if it % 10 == 0 and e["spawn_ratio_max"] > 0:
            assert e["tau"] * e["spawn_ratio_max"] <= 1.0 + 1e-15
    assert taus[-1] < 0.05
    # Hubbard hopping: |H| = t and p_gen = 1 / (number of hops), so the ratio is at most 16 on the 8-site ring
    assert 0 < r.estimators()["spawn_ratio_max"] <= 16.0 + 1e-12


def test_without_the_search_tau_is_constant():
    r = O.Run(O.System.hubbard(), O.make_qmc(tau=0.01, initial_shift=-4.0))
    for _ in range(5):
        r.step(10)
        e = r.estimators()
        assert e["tau"] == 0.01 and e["spawn_ratio_max"] == 0.0


def test_death_bound_uses_the_largest_diagonal_of_the_last_death_step():
    # Hubbard ring from tau = 0.05: at the first shift update the death bound
    # 1 / (max K_ii - S) is the binding one (the spawn bound is 1/16). K_ii is
    # recomputed here from the list the last death step acted on.
    s = O.System.hubbard()
    r = O.Run(s, O.make_qmc(tau=0.05, initial_shift=-4.0, tau_search=1))
    r.step(9)
    keys, pops = r.export()  # the list iteration 10 starts from
    kii = max(s.diag(k) - s.H00 for k, p in zip(keys, pops) if p != 0)
    r.step(1)
    e = r.estimators()
    expect = min(0.05, 1.0 / e["spawn_ratio_max"], 1.0 / (kii - e["shift"]))
    assert 1.0 / (kii - e["shift"]) < 1.0 / e["spawn_ratio_max"]
    assert e["tau"] == expect
