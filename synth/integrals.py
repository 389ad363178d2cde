"""Seeded molecular-like integrals for the ab initio Hamiltonian (Sec. II.A.1).

The paper's workloads are active spaces whose integrals come from a quantum
chemistry package; those integral files are not available here, so seeded
Gaussian integrals of the same orbital counts stand in for them.

Recipe (reading of the workload description):
  * rng = numpy.random.default_rng(seed) (PCG64);
  * h: the upper triangle including the diagonal is drawn row-major as N(0,1),
    divided by sqrt(K), and mirrored;
  * for k = 0..15: a symmetric matrix L^k is drawn the same way and scaled by 0.1;
  * g_pqrs = sum_k L^k_pq L^k_rs (chemists' notation (pq|rs)); this has the full
    8-fold permutational symmetry and is positive semi-definite as a K^2 x K^2
    matrix.
"""

import numpy as np


def _sym_upper(rng, K):
    iu = np.triu_indices(K)
    m = np.zeros((K, K))
    m[iu] = rng.standard_normal(len(iu[0]))
    return m + np.triu(m, 1).T


def make_integrals(K, seed=0, rank=16, g_scale=0.1):
    """Return (h[K,K], g[K,K,K,K]) drawn by the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    h = _sym_upper(rng, K) / np.sqrt(K)
    g = np.zeros((K, K, K, K))
    for _ in range(rank):
        lk = _sym_upper(rng, K) * g_scale
        g += np.einsum("pq,rs->pqrs", lk, lk)
    return h, g


def hubbard_integrals(K, t, U, periodic=False):
    """Hubbard chain as (h, g): h = -t on nearest neighbours, g_pppp = U."""
    h = np.zeros((K, K))
    for p in range(K - 1):
        h[p, p + 1] = h[p + 1, p] = -t
    if periodic and K > 2:
        h[0, K - 1] = h[K - 1, 0] = -t
    g = np.zeros((K, K, K, K))
    for p in range(K):
        g[p, p, p, p] = U
    return h, g
