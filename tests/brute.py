"""Brute-force references for the oracle pins (test helpers, pure Python/numpy).

Nothing here reuses the oracle's Slater-Condon rules: matrices are built by
applying the second-quantised operators a+_A a_P and a+_A a+_B a_Q a_P to bit
strings with Jordan-Wigner signs, exactly as the operators are defined.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def annihilate(bits: int, P: int):
    if not (bits >> P) & 1:
        return None
    sign = -1 if bin(bits & ((1 << P) - 1)).count("1") & 1 else 1
    return sign, bits ^ (1 << P)


def create(bits: int, A: int):
    if (bits >> A) & 1:
        return None
    sign = -1 if bin(bits & ((1 << A) - 1)).count("1") & 1 else 1
    return sign, bits | (1 << A)


def occupied(bits: int):
    out, P = [], 0
    while bits >> P:
        if (bits >> P) & 1:
            out.append(P)
        P += 1
    return out


def all_dets(n_spatial: int, n_alpha: int, n_beta: int):
    """Every determinant with the given spin populations (P = 2p + sigma)."""
    dets = []
    for a in itertools.combinations(range(n_spatial), n_alpha):
        for b in itertools.combinations(range(n_spatial), n_beta):
            bits = 0
            for p in a:
                bits |= 1 << (2 * p)
            for p in b:
                bits |= 1 << (2 * p + 1)
            dets.append(bits)
    return sorted(dets)


def second_quantised_matrix(dets, n_so, h1=None, g=None, diag_fn=None):
    """<D_i| sum_AP h_AP a+_A a_P + 1/2 sum <AB|PQ> a+_A a+_B a_Q a_P (+ diag_fn) |D_j>."""
    index = {d: i for i, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for j, d in enumerate(dets):
        occ = occupied(d)
        if diag_fn is not None:
            H[j, j] += diag_fn(d)
        if h1 is not None:
            for P in occ:
                r1 = annihilate(d, P)
                for A in range(n_so):
                    v = h1(A, P)
                    if v == 0.0:
                        continue
                    r2 = create(r1[1], A)
                    if r2 is None or r2[1] not in index:
                        continue
                    H[index[r2[1]], j] += v * r1[0] * r2[0]
        if g is not None:
            for P in occ:
                r1 = annihilate(d, P)
                for Q in occ:
                    if Q == P:
                        continue
                    r2 = annihilate(r1[1], Q)
                    for B in range(n_so):
                        r3 = create(r2[1], B)
                        if r3 is None:
                            continue
                        for A in range(n_so):
                            v = g(A, B, P, Q)
                            if v == 0.0:
                                continue
                            r4 = create(r3[1], A)
                            if r4 is None or r4[1] not in index:
                                continue
                            H[index[r4[1]], j] += 0.5 * v * r1[0] * r2[0] * r3[0] * r4[0]
    return H


def apply_h(d, n_so, h1=None, g=None, diag_fn=None):
    """H|d> as a dict {determinant: amplitude} (same operator definition as above)."""
    out = {}

    def add(k, v):
        out[k] = out.get(k, 0.0) + v

    occ = occupied(d)
    if diag_fn is not None:
        add(d, diag_fn(d))
    if h1 is not None:
        for P in occ:
            r1 = annihilate(d, P)
            for A in range(n_so):
                v = h1(A, P)
                if v == 0.0:
                    continue
                r2 = create(r1[1], A)
                if r2 is not None:
                    add(r2[1], v * r1[0] * r2[0])
    if g is not None:
        for P in occ:
            r1 = annihilate(d, P)
            for Q in occ:
                if Q == P:
                    continue
                r2 = annihilate(r1[1], Q)
                for B in range(n_so):
                    r3 = create(r2[1], B)
                    if r3 is None:
                        continue
                    for A in range(n_so):
                        v = g(A, B, P, Q)
                        if v == 0.0:
                            continue
                        r4 = create(r3[1], A)
                        if r4 is not None:
                            add(r4[1], 0.5 * v * r1[0] * r2[0] * r3[0] * r4[0])
    return out


def ueg_operators(rs, ecut, nel):
    kv = ueg_plane_waves(ecut)
    L = rs * (4.0 * math.pi * nel / 3.0) ** (1.0 / 3.0)
    kk = (2.0 * math.pi / L) ** 2

    def h1(A, P):
        if A != P:
            return 0.0
        n = kv[P >> 1]
        return 0.5 * kk * (n[0] ** 2 + n[1] ** 2 + n[2] ** 2)

    def g(A, B, P, Q):
        if (A & 1) != (P & 1) or (B & 1) != (Q & 1):
            return 0.0
        a, b, p, q = (kv[X >> 1] for X in (A, B, P, Q))
        if any(a[i] + b[i] != p[i] + q[i] for i in range(3)):
            return 0.0
        d2 = sum((p[i] - a[i]) ** 2 for i in range(3))
        if d2 == 0:
            return 0.0
        return 4.0 * math.pi / (L ** 3 * kk * d2)

    return kv, h1, g, L


def hubbard_matrix(n_sites, n_alpha, n_beta, t, U, periodic=True):
    dets = all_dets(n_sites, n_alpha, n_beta)
    bonds = set()
    for p in range(n_sites):
        for q in (p - 1, p + 1):
            if 0 <= q < n_sites or periodic:
                bonds.add((p, q % n_sites))

    def h1(A, P):
        if (A & 1) != (P & 1):
            return 0.0
        return -t if (A >> 1, P >> 1) in bonds else 0.0

    def diag(bits):
        return U * sum(1 for p in range(n_sites) if (bits >> (2 * p)) & 1 and (bits >> (2 * p + 1)) & 1)

    return dets, second_quantised_matrix(dets, 2 * n_sites, h1=h1, diag_fn=diag)


def ueg_plane_waves(ecut):
    c = int(math.isqrt(ecut))
    pw = [(x * x + y * y + z * z, x, y, z) for x in range(-c, c + 1) for y in range(-c, c + 1)
          for z in range(-c, c + 1) if x * x + y * y + z * z <= ecut]
    pw.sort()
    return [(x, y, z) for _, x, y, z in pw]


def ueg_matrix(rs, ecut, n_alpha, n_beta):
    """Plane-wave UEG in a cubic box, Coulomb 4 pi/(L^3 k^2), k = 0 term dropped."""
    kv = ueg_plane_waves(ecut)
    M = len(kv)
    N = n_alpha + n_beta
    L = rs * (4.0 * math.pi * N / 3.0) ** (1.0 / 3.0)
    kk = (2.0 * math.pi / L) ** 2
    dets = all_dets(M, n_alpha, n_beta)

    def h1(A, P):
        if A != P:
            return 0.0
        n = kv[P >> 1]
        return 0.5 * kk * (n[0] ** 2 + n[1] ** 2 + n[2] ** 2)

    def g(A, B, P, Q):
        if (A & 1) != (P & 1) or (B & 1) != (Q & 1):
            return 0.0
        a, b, p, q = (kv[X >> 1] for X in (A, B, P, Q))
        if any(a[i] + b[i] != p[i] + q[i] for i in range(3)):
            return 0.0
        d2 = sum((p[i] - a[i]) ** 2 for i in range(3))
        if d2 == 0:
            return 0.0
        return 4.0 * math.pi / (L ** 3 * kk * d2)

    return dets, second_quantised_matrix(dets, 2 * M, h1=h1, g=g), L


def molecular_matrix(h, eri, n_alpha, n_beta):
    n = h.shape[0]
    dets = all_dets(n, n_alpha, n_beta)

    def h1(A, P):
        return float(h[A >> 1, P >> 1]) if (A & 1) == (P & 1) else 0.0

    def g(A, B, P, Q):
        if (A & 1) != (P & 1) or (B & 1) != (Q & 1):
            return 0.0
        return float(eri[A >> 1, P >> 1, B >> 1, Q >> 1])

    return dets, second_quantised_matrix(dets, 2 * n, h1=h1, g=g)


def reblock(x):
    """Flyvbjerg-Petersen blocking: (mean, standard error at the plateau)."""
    x = np.asarray(x, float)
    mean = x.mean()
    errs = []
    while len(x) >= 16:
        errs.append(x.std(ddof=1) / math.sqrt(len(x)))
        if len(x) % 2:
            x = x[:-1]
        x = 0.5 * (x[0::2] + x[1::2])
    return mean, max(errs) if errs else float("nan")


def key_words(bits: int, W: int):
    return np.array([(bits >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(W)], dtype=np.uint64)


def words_int(words) -> int:
    return sum(int(w) << (64 * i) for i, w in enumerate(words))
