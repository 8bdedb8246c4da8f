"""Exhaustive enumeration of the excitation generators' choice trees.

For a determinant D every branch of a generator is driven with forced random
words (the smallest word that maps to each discrete choice, the midpoint of
each continuous interval). The branch measures must sum to one (null draws
included), the measure reaching each child must equal the p_gen the generator
reports, and every determinant connected to D by H must be reachable
(paper Sec. 2.4: random selection of a connected state with a known
probability; heat-bath weights, Sec. 2.1).
"""
import math

import numpy as np

import brute
from paper_1811_11679_amd import synth

TWO32 = 1 << 32


def forced(k, n):
    """smallest 32-bit word w with floor(w n / 2^32) = k, and the count of such words"""
    lo = -((-k * TWO32) // n)
    hi = -((-(k + 1) * TWO32) // n)
    return lo, hi - lo


def words_for_u(u):
    m = int(u * 2.0**53)
    return m >> 21, (m & ((1 << 21) - 1)) << 11


def check_tree(branches, pgen, conn):
    total = sum(p for p, _ in branches)
    assert abs(total - 1.0) < 1e-12
    per_child = {}
    for p, c in branches:
        if c is not None:
            per_child[c] = per_child.get(c, 0.0) + p
    for c, p in per_child.items():
        assert abs(p - pgen[c]) <= 2e-6 * pgen[c], (p, pgen[c])
    missing = set(conn) - set(per_child)
    assert not missing


def test_hubbard_generator_tree(oracle_mod):
    for periodic in (True, False):
        s = oracle_mod.System.hubbard(n_sites=8, periodic=periodic, n_alpha=4, n_beta=3)
        dets = brute.all_dets(8, 4, 3)
        rng = np.random.default_rng(0)
        bonds = {(p, (p + d) % 8) for p in range(8) for d in (-1, 1) if periodic or 0 <= p + d < 8}
        h1 = lambda A, P: -1.0 if (A & 1) == (P & 1) and (A >> 1, P >> 1) in bonds else 0.0
        for i in rng.choice(len(dets), size=40, replace=False):
            d = dets[i]
            key = brute.key_words(d, 1)
            conn = {x for x, v in brute.apply_h(d, 16, h1=h1).items() if x != d and v != 0.0}
            nv = len(conn)
            branches, pg = [], {}
            for k in range(nv):
                w, cnt = forced(k, nv)
                r = s.exgen(oracle_mod.EXGEN_HUB, key, [w])
                c = brute.words_int(r[0])
                branches.append((cnt / TWO32, c))
                pg[c] = r[1]
                assert r[2] == brute.apply_h(d, 16, h1=h1)[c]
            check_tree(branches, pg, conn)


def _ueg_tree(oracle_mod, s, d, W, rs, ecut):
    kv, h1, g, L = brute.ueg_operators(rs, ecut, s.nel)
    key = brute.key_words(d, W)
    occ = brute.occupied(d)
    N = len(occ)
    npairs = N * (N - 1) // 2
    M = s.n_spatial
    branches, pg = [], {}
    k = 0
    for i in range(N):
        for j in range(i + 1, N):
            wk, ck = forced(k, npairs)
            same = (occ[i] & 1) == (occ[j] & 1)
            na = M if same else 2 * M
            for a in range(na):
                wa, ca = forced(a, na)
                r = s.exgen(oracle_mod.EXGEN_UEG, key, [wk, wa])
                p = (ck / TWO32) * (ca / TWO32)
                if r is None:
                    branches.append((p, None))
                else:
                    c = brute.words_int(r[0])
                    branches.append((p, c))
                    pg[c] = r[1]
                    assert abs(r[2] - s.hij(r[0], key)) == 0.0
            k += 1
    col = brute.apply_h(d, 2 * M, h1=h1, g=g)
    conn = {x for x, v in col.items() if x != d and v != 0.0}
    for c in pg:
        assert abs(s.hij(brute.key_words(c, W), key) - col.get(c, 0.0)) < 1e-13
    check_tree(branches, pg, conn)


def test_ueg_generator_tree_small(oracle_mod):
    s = oracle_mod.System.ueg(rs=1.0, ecut=2, n_alpha=3, n_beta=2)
    dets = brute.all_dets(19, 3, 2)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(dets), size=6, replace=False):
        _ueg_tree(oracle_mod, s, dets[i], 1, 1.0, 2)


def test_ueg_generator_tree_two_words(oracle_mod):
    # 57 plane waves (W = 2): the reference and a random double of it
    s = oracle_mod.System.ueg(rs=1.0, ecut=5, n_alpha=3, n_beta=3)
    ref = brute.words_int(s.ref)
    _ueg_tree(oracle_mod, s, ref, 2, 1.0, 5)
    d = ref & ~(1 << 0) & ~(1 << 3)
    d |= (1 << 100) | (1 << 113)
    _ueg_tree(oracle_mod, s, d, 2, 1.0, 5)


def _hb_tables(h, eri, n_so):
    """independent numpy weights |<AB|PQ> - <AB|QP>| per allowed (P<Q, A<B)"""
    def g(A, B, P, Q):
        x = eri[A >> 1, P >> 1, B >> 1, Q >> 1] if (A & 1) == (P & 1) and (B & 1) == (Q & 1) else 0.0
        y = eri[A >> 1, Q >> 1, B >> 1, P >> 1] if (A & 1) == (Q & 1) and (B & 1) == (P & 1) else 0.0
        return x - y
    tab = {}
    for P in range(n_so):
        for Q in range(P + 1, n_so):
            ent = []
            for A in range(n_so):
                for B in range(A + 1, n_so):
                    if len({A, B, P, Q}) < 4 or (A & 1) + (B & 1) != (P & 1) + (Q & 1):
                        continue
                    ent.append((A, B, abs(g(A, B, P, Q))))
            tab[(P, Q)] = ent
    return tab


def test_heatbath_generator_tree(oracle_mod):
    ps = 0.1
    h, eri = synth.molecular_integrals(n_orb=6, n_chol=8, seed=3, sigma_h=0.2, sigma_l=0.4)
    s = oracle_mod.System.molecular(h, eri, 3, 2)
    n_so = 12
    tab = _hb_tables(h, eri, n_so)
    hb1 = lambda A, P: float(h[A >> 1, P >> 1]) if (A & 1) == (P & 1) else 0.0
    gb = lambda A, B, P, Q: (float(eri[A >> 1, P >> 1, B >> 1, Q >> 1])
                             if (A & 1) == (P & 1) and (B & 1) == (Q & 1) else 0.0)
    dets = brute.all_dets(6, 3, 2)
    rng = np.random.default_rng(2)
    for i in rng.choice(len(dets), size=8, replace=False):
        d = dets[i]
        key = brute.key_words(d, 1)
        occ = brute.occupied(d)
        N = len(occ)
        branches, pg = [], {}
        # singles: d < p_single, uniform occupied, uniform empty orbital of that spin
        for e in range(N):
            we, ce = forced(e, N)
            sg = occ[e] & 1
            nv = 6 - (3 if sg == 0 else 2)
            for a in range(nv):
                wa, ca = forced(a, nv)
                r = s.exgen(oracle_mod.EXGEN_HEATBATH, key, [0, 0, we, wa], p_single=ps)
                p = ps * (ce / TWO32) * (ca / TWO32)
                c = brute.words_int(r[0])
                branches.append((p, c))
                pg[c] = r[1]
        # doubles
        pairs = [(occ[i], occ[j]) for i in range(N) for j in range(i + 1, N)]
        S = [sum(w for _, _, w in tab[pq]) for pq in pairs]
        T = sum(S)
        cum = 0.0
        for pq, Sk in zip(pairs, S):
            if Sk == 0.0:
                continue
            u = (cum + 0.5 * Sk) / T
            cum += Sk
            w4, w5 = words_for_u(u)
            c2 = 0.0
            for A, B, w in tab[pq]:
                if w == 0.0:
                    continue
                u2 = (c2 + 0.5 * w) / Sk
                c2 += w
                w6, w7 = words_for_u(u2)
                r = s.exgen(oracle_mod.EXGEN_HEATBATH, key,
                            [0xFFFFFFFF, 0xFFFFFFFF, 0, 0, w4, w5, w6, w7], p_single=ps)
                p = (1.0 - ps) * w / T
                if (d >> A) & 1 or (d >> B) & 1:
                    assert r is None
                    branches.append((p, None))
                else:
                    c = brute.words_int(r[0])
                    assert c == (d & ~(1 << pq[0]) & ~(1 << pq[1])) | (1 << A) | (1 << B)
                    branches.append((p, c))
                    pg[c] = r[1]
                    assert abs(r[1] - p) <= 1e-12 * p  # heat-bath: p_gen proportional to |H|
        col = brute.apply_h(d, n_so, h1=hb1, g=gb)
        conn = {x for x, v in col.items() if x != d and abs(v) > 1e-14}
        for c in pg:
            assert abs(s.hij(brute.key_words(c, 1), key) - col.get(c, 0.0)) < 1e-12
        check_tree(branches, pg, conn)
