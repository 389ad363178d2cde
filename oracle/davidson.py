"""Textbook Davidson eigensolver (Davidson 1975) with a diagonal preconditioner.

The paper's sweeps solve the two-site eigenproblem with Davidson (Listing 1 caps
it at 30 iterations with a 1e-10 threshold).  One step, given an orthonormal
basis V (rows v_0..v_{k-1}) and S = H V:

  1. projected matrix G_ij = v_i . s_j, symmetrised as (G + G^T) / 2;
  2. lowest eigenpair (theta, y) of G; y is normalised and its largest-magnitude
     entry is made positive;
  3. Ritz vector x = sum_j y_j v_j, its image hx = sum_j y_j s_j, residual
     r = hx - theta x and ||r||;
  4. correction t_e = r_e / (theta - d_e), with |theta - d_e| raised to `guard`
     (keeping its sign, + for zero) where it is smaller;
  5. t orthogonalised against V by classical Gram-Schmidt, twice, then normalised.

Restart: when the basis is full, V <- [x], S <- [hx].
"""

import numpy as np


def ritz(V, S):
    G = V @ S.T
    G = 0.5 * (G + G.T)
    w, U = np.linalg.eigh(G)
    y = U[:, 0].copy()
    j = int(np.argmax(np.abs(y)))
    if y[j] < 0:
        y = -y
    return float(w[0]), y, G


def correction(r, theta, diag, guard):
    den = theta - diag
    small = np.abs(den) < guard
    den = np.where(small, np.where(den < 0, -guard, guard), den)
    return r / den


def orthonormalise(t, V):
    for _ in range(2):
        t = t - V.T @ (V @ t)
    nrm = float(np.linalg.norm(t))
    return t / nrm if nrm > 0 else t, nrm


def step(V, S, diag, guard=1e-8):
    theta, y, _ = ritz(V, S)
    x = y @ V
    hx = y @ S
    r = hx - theta * x
    rnorm = float(np.linalg.norm(r))
    t = correction(r, theta, diag, guard)
    t, tnorm = orthonormalise(t, V)
    return theta, rnorm, x, hx, t, tnorm


def solve(matvec, x0, diag, tol=1e-8, max_iter=200, kmax=24, guard=1e-8):
    """Lowest eigenpair; returns (theta, x, n_matvec, rnorm)."""
    v = x0 / np.linalg.norm(x0)
    V = v[None, :]
    S = matvec(v)[None, :]
    nmv = 1
    theta, rnorm, x = None, None, v
    for _ in range(max_iter):
        theta, rnorm, x, hx, t, tnorm = step(V, S, diag, guard)
        if rnorm < tol:
            break
        if V.shape[0] >= kmax:
            V, S = x[None, :] / np.linalg.norm(x), hx[None, :] / np.linalg.norm(x)
            t, tnorm = orthonormalise(correction(hx - theta * x, theta, diag, guard), V)
        V = np.vstack([V, t])
        S = np.vstack([S, matvec(t)])
        nmv += 1
    return theta, x, nmv, rnorm
