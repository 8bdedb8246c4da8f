"""Oracle density-matrix methods pinned to their propagation equations and to
exact diagonalisation (paper Sec. 2.3, eqs. dmqmc and ipdmqmc; Sec. 2.4).

States are pairs (D_i, D_j) holding rho_ij: a key of the bra's words then
the ket's. With K = H - H_00 and a fixed shift S:

* DMQMC, one step of the symmetrised Bloch equation:
    E[rho'] = rho - (dbeta / 2)(K rho + rho K) + dbeta S rho;
* IP-DMQMC (H^0 the diagonal part of H), one step of df/dtau = H^0 f - f H:
    E[f'] = f + dtau (K^0 f - f K + S f);
* a beta-loop average of Tr(rho H) and Tr(rho) equals the same linear map
  applied n times to the starting matrix (each step is unbiased and linear),
  and Tr(rho H) / Tr(rho) from rho(0) = I approaches the thermal energy of
  exact diagonalisation, sum_a E_a e^{-beta E_a} / sum_a e^{-beta E_a}.
"""
import numpy as np
import pytest

import brute


def _pair_key(bra, ket, W):
    return np.concatenate([brute.key_words(bra, W), brute.key_words(ket, W)])


def _matrix_from_export(keys, pops, index, W):
    n = len(index)
    m = np.zeros((n, n))
    for kk, pp in zip(keys, pops):
        m[index[brute.words_int(kk[:W])], index[brute.words_int(kk[W:])]] = pp
    return m


def _hubbard4(O):
    # 3 + 2 electrons on a 4-site ring (24 determinants): the reference holds a
    # double occupancy, so H_00 = U and K = H - H_00 differs from H
    s = O.System.hubbard(n_sites=4, periodic=True, t=1.0, U=4.0, n_alpha=3, n_beta=2)
    dets, Hb = brute.hubbard_matrix(4, 3, 2, 1.0, 4.0)
    assert s.H00 == 4.0
    return s, dets, Hb


def _one_step(O, s, dets, Hb, state, kw, trials, method):
    W = s.W
    index = {d: i for i, d in enumerate(dets)}
    n = len(dets)
    rho = np.zeros((n, n))
    for (i, j), p in state.items():
        rho[i, j] = p
    keys = np.stack([_pair_key(dets[i], dets[j], W) for (i, j) in state])
    pops = np.array(list(state.values()), np.int32)
    S, tau = kw.get("initial_shift", 0.0), kw["tau"]
    K = Hb - s.H00 * np.eye(n)
    if method == O.DMQMC:
        expect = rho - 0.5 * tau * (K @ rho + rho @ K) + tau * S * rho
    else:
        K0 = np.diag(np.diag(K))
        expect = rho + tau * (K0 @ rho - rho @ K + S * rho)
    acc = np.zeros((n, n))
    acc2 = np.zeros((n, n))
    for seed in range(trials):
        r = O.Run(s, O.make_qmc(seed=500 + seed, method=method, **kw))
        r.import_walkers(keys, pops, shift=S, iteration=3)
        r.step(1)
        k2, p2 = r.export()
        v = _matrix_from_export(k2, p2, index, W)
        acc += v
        acc2 += v * v
    mean = acc / trials
    se = np.sqrt(np.maximum(acc2 / trials - mean ** 2, 0.0) / trials)
    touched = (se > 0) | (np.abs(expect) > 0)
    z = np.abs(mean - expect) / np.maximum(se, 1e-9)
    assert z[touched].max() < 5.5, z[touched].max()
    assert (se > 0).sum() >= 20
    return mean


def test_dmqmc_one_step_expectation_integer(oracle_mod):
    O = oracle_mod
    s, dets, Hb = _hubbard4(O)
    rng = np.random.default_rng(4)
    n = len(dets)
    state = {(int(i), int(j)): int(rng.integers(-40, 40)) or 9
             for i, j in zip(rng.integers(0, n, 14), rng.integers(0, n, 14))}
    for i in range(0, n, 7):
        state[(i, i)] = 30
    mean = _one_step(O, s, dets, Hb, state, dict(tau=0.05, excit_gen=O.EXGEN_HUB, initial_shift=-0.4), 3000,
                     O.DMQMC)
    # both ends spawn: rows and columns of the occupied pairs change
    assert np.count_nonzero(mean) > len(state)


def test_dmqmc_one_step_expectation_fixed_point(oracle_mod):
    O = oracle_mod
    s, dets, Hb = _hubbard4(O)
    rng = np.random.default_rng(5)
    n = len(dets)
    state = {(int(i), int(j)): int(rng.integers(-3000, 3000)) or 77
             for i, j in zip(rng.integers(0, n, 10), rng.integers(0, n, 10))}
    _one_step(O, s, dets, Hb, state, dict(tau=0.03, excit_gen=O.EXGEN_HUB, fixed_point_bits=8, spawn_cutoff=0.1,
                                          initial_shift=0.3), 2500, O.DMQMC)


def test_ipdmqmc_one_step_expectation(oracle_mod):
    O = oracle_mod
    s, dets, Hb = _hubbard4(O)
    rng = np.random.default_rng(6)
    n = len(dets)
    state = {(int(i), int(j)): int(rng.integers(-50, 50)) or 13
             for i, j in zip(rng.integers(0, n, 14), rng.integers(0, n, 14))}
    mean = _one_step(O, s, dets, Hb, state, dict(tau=0.05, excit_gen=O.EXGEN_HUB, initial_shift=-0.2), 3000,
                     O.IPDMQMC)
    # only the ket end spawns: no row outside the occupied bras changes
    rows = {i for (i, _) in state}
    assert all(np.all(mean[i] == 0) for i in range(n) if i not in rows)


def _beta_loops(O, s, dets, keys, pops, kw, n_steps, loops):
    num = np.zeros((loops, n_steps))
    den = np.zeros((loops, n_steps))
    for L in range(loops):
        r = O.Run(s, O.make_qmc(seed=9000 + L, **kw))
        r.import_walkers(keys, pops, shift=kw.get("initial_shift", 0.0), iteration=0)
        for t in range(n_steps):
            r.step(1)
            e = r.estimators()
            num[L, t] = e["proj_numerator"]
            den[L, t] = e["ref_pop_units"] * 2.0 ** -kw.get("fixed_point_bits", 0)
    return num, den


def test_dmqmc_beta_loops_sample_the_thermal_energy(oracle_mod):
    O = oracle_mod
    s, dets, Hb = _hubbard4(O)
    n, W = len(dets), s.W
    c, tau, n_steps, loops = 8, 0.02, 50, 300
    keys = np.stack([_pair_key(d, d, W) for d in dets])
    pops = np.full(n, c, np.int32)
    kw = dict(tau=tau, excit_gen=O.EXGEN_HUB, method=O.DMQMC, target_population=1e12)
    num, den = _beta_loops(O, s, dets, keys, pops, kw, n_steps, loops)
    # exact expectation of the same linear map: eigenvalues of K, rho_0 = c I
    E, _ = np.linalg.eigh(Hb)
    lam = 1.0 - tau * (E - s.H00)
    for t in (9, 24, 49):
        w = lam ** (t + 1)
        exp_num, exp_den = c * np.sum(w * E), c * np.sum(w)
        for x, ex in ((num[:, t], exp_num), (den[:, t], exp_den)):
            se = x.std(ddof=1) / np.sqrt(loops)
            assert abs(x.mean() - ex) < 4.5 * se + 1e-9, (t, x.mean(), ex, se)
    # the ratio of the averages against exact diagonalisation (thermal energy)
    beta = tau * n_steps
    e_ed = np.sum(E * np.exp(-beta * E)) / np.sum(np.exp(-beta * E))
    ratio = num[:, -1].mean() / den[:, -1].mean()
    e_disc = np.sum(lam ** n_steps * E) / np.sum(lam ** n_steps)
    assert abs(e_disc - e_ed) < 0.05  # first-order time step: O(dbeta)
    assert abs(ratio - e_ed) < 0.1, (ratio, e_ed)


def test_ipdmqmc_beta_loops_follow_the_interaction_picture_map(oracle_mod):
    O = oracle_mod
    s, dets, Hb = _hubbard4(O)
    n, W = len(dets), s.W
    tau, n_steps, loops = 0.02, 40, 300
    beta = tau * n_steps
    K = Hb - s.H00 * np.eye(n)
    k0 = np.diag(K)
    # f(0) = e^{-beta H^0} up to a constant, rounded to whole walkers
    f0 = np.rint(60.0 * np.exp(-beta * (k0 - k0.min()))).astype(np.int32)
    keep = f0 > 0
    keys = np.stack([_pair_key(d, d, W) for d, k in zip(dets, keep) if k])
    pops = f0[keep]
    kw = dict(tau=tau, excit_gen=O.EXGEN_HUB, method=O.IPDMQMC, target_population=1e12)
    num, den = _beta_loops(O, s, dets, keys, pops, kw, n_steps, loops)
    f = np.diag(f0.astype(float))
    K0 = np.diag(k0)
    for t in range(n_steps):
        f = f + tau * (K0 @ f - f @ K)
        if t in (19, n_steps - 1):
            exp_num, exp_den = np.trace(f @ Hb), np.trace(f)
            for x, ex in ((num[:, t], exp_num), (den[:, t], exp_den)):
                se = x.std(ddof=1) / np.sqrt(loops)
                assert abs(x.mean() - ex) < 4.5 * se + 1e-9, (t, x.mean(), ex, se)
    # at tau = beta, f is a sample of rho(beta): the thermal energy
    E, _ = np.linalg.eigh(Hb)
    e_ed = np.sum(E * np.exp(-beta * E)) / np.sum(np.exp(-beta * E))
    assert abs(num[:, -1].mean() / den[:, -1].mean() - e_ed) < 0.1


def test_density_matrix_runs_refuse_what_they_do_not_support(oracle_mod):
    O = oracle_mod
    s, _, _ = _hubbard4(O)
    for bad in (dict(initiator=1), dict(ss_size=10), dict(tau_search=1), dict(method=3)):
        kw = dict(tau=0.01, excit_gen=O.EXGEN_HUB, method=O.DMQMC)
        kw.update(bad)
        with pytest.raises(ValueError):
            O.Run(s, O.make_qmc(**kw))
