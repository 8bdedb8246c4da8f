"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws numbers (integral arrays, run parameters). It holds none
of the FCIQMC arithmetic: no matrix elements, no excitation generation, no
propagation. Both the oracle and the HIP library receive its arrays as inputs.

Molecular-like Hamiltonian (stands in for the all-electron molecular systems of
the paper's Results section, whose integral files are not available):

* one-electron h_pq: diagonal eps_p ~ U[-2, 2] Ha sorted ascending (so the
  aufbau determinant fills the lowest orbitals), off-diagonal h_pq = h_qp with
  standard deviation 0.05 Ha;
* two-electron (pq|rs) = sum_K L^K_pq L^K_rs (chemists' notation), with
  L^K_pq = L^K_qp = g * exp(-|p - q| / 4), g ~ N(0, sigma_L^2); this
  factorised form is positive semi-definite and has the 8-fold permutational
  symmetry of real orbitals.
"""
from __future__ import annotations

import numpy as np


def molecular_integrals(n_orb: int = 30, n_chol: int = 60, seed: int = 7,
                        sigma_h: float = 0.05, sigma_l: float = 0.1,
                        decay: float = 4.0):
    """Return (h1[n,n], eri[n,n,n,n]) as C-contiguous float64 arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.sort(rng.uniform(-2.0, 2.0, size=n_orb))
    h = rng.normal(0.0, sigma_h, size=(n_orb, n_orb))
    h = np.triu(h, 1)
    h = h + h.T
    h[np.diag_indices(n_orb)] = eps
    idx = np.arange(n_orb)
    envelope = np.exp(-np.abs(idx[:, None] - idx[None, :]) / decay)
    chol = np.empty((n_chol, n_orb, n_orb))
    for k in range(n_chol):
        g = rng.normal(0.0, sigma_l, size=(n_orb, n_orb))
        g = np.triu(g) + np.triu(g, 1).T
        chol[k] = g * envelope
    eri = np.einsum("kpq,krs->pqrs", chol, chol, optimize=True)
    # symmetrise exactly so that every permutation reads the same bits
    eri = 0.5 * (eri + eri.transpose(1, 0, 2, 3))
    eri = 0.5 * (eri + eri.transpose(0, 1, 3, 2))
    eri = 0.5 * (eri + eri.transpose(2, 3, 0, 1))
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def batched_ueg_draws(n_replicas: int = 64, seed: int = 7,
                      rs_choices=(0.5, 1.0, 2.0, 4.0),
                      basis_choices=(19, 27, 57, 123),
                      target_lo: float = 1e5, target_hi: float = 2e6):
    """Per-replica (rs, n_plane_waves, target) for the batched UEG workload.

    rs and the basis size are drawn uniformly from the given sets, the target
    population log-uniformly in [target_lo, target_hi].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rs = rng.choice(np.asarray(rs_choices), size=n_replicas)
    m = rng.choice(np.asarray(basis_choices), size=n_replicas)
    tgt = np.exp(rng.uniform(np.log(target_lo), np.log(target_hi), size=n_replicas))
    return [(float(a), int(b), float(np.round(c))) for a, b, c in zip(rs, m, tgt)]


def random_walker_state(n_dets: int, sample_det, seed: int = 11,
                        max_abs: int = 2000):
    """Draw a seeded list of distinct determinants with nonzero populations.

    ``sample_det(rng)`` must return one determinant as a tuple of uint64
    words; it is supplied by the caller (the test or benchmark) so this module
    stays free of any system-specific arithmetic.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    seen = {}
    while len(seen) < n_dets:
        d = tuple(int(x) for x in sample_det(rng))
        if d in seen:
            continue
        p = int(rng.integers(1, max_abs + 1)) * (1 if rng.random() < 0.7 else -1)
        seen[d] = p
    keys = np.array(list(seen.keys()), dtype=np.uint64)
    pops = np.array(list(seen.values()), dtype=np.int32)
    return keys, pops
