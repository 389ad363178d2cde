"""Hubbard-Holstein model of Listing 1, solved by exact diagonalisation.

Reading of the listing's terms (each term string is a product of the printed
on-site matrices; c, d, C, D are a+_alpha, a_alpha, a+_beta, a_beta; E, F are
b+ and b on a phonon site truncated to N_PH levels):
  * "cd" and "CD" over index quadruples [i, i+1, i+1, i] with coefficient -1:
    nearest-neighbour hopping of each spin in both directions;
  * "cdCD" at [i, i, i, i] with coefficient U: U n_alpha n_beta;
  * "EF" with coefficient omega: omega b+ b on every phonon site;
  * "cdE", "cdF", "CDE", "CDF" at [i, i, i + n_elec_sites] with coefficient g:
    g (n_alpha + n_beta)(b+ + b), electron site i coupled to phonon site i.
The printed ground-state energy for N = 4 electrons, 2Sz = 0 is -6.956893.
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import fock


def ground_energy(n_sites=4, n_ph=11, U=2.0, omega=0.25, g=0.5, n_elec=4, twosz=0):
    K = n_sites
    h = np.zeros((K, K))
    for i in range(K - 1):
        h[i, i + 1] = h[i + 1, i] = -1.0
    gg = np.zeros((K, K, K, K))
    for i in range(K):
        gg[i, i, i, i] = U
    dets = fock.sector_dets(K, n_elec, twosz)
    Hel = fock.hamiltonian(h, gg, dets).toarray()
    ne = len(dets)
    nocc = np.array([[((d >> (2 * i)) & 1) + ((d >> (2 * i + 1)) & 1) for i in range(K)] for d in dets],
                    dtype=float)  # (ne, K)
    bdag = np.diag(np.sqrt(np.arange(1, n_ph)), k=-1)
    x = bdag + bdag.T
    nph = np.arange(n_ph, dtype=float)
    shape = (ne,) + (n_ph,) * K

    def matvec(v):
        t = v.reshape(shape)
        out = np.tensordot(Hel, t, axes=([1], [0]))
        for i in range(K):
            # omega b+_i b_i
            sh = [1] * (K + 1)
            sh[i + 1] = n_ph
            out += omega * t * nph.reshape(sh)
            # g n_i (b+_i + b_i)
            xt = np.moveaxis(np.tensordot(x, t, axes=([1], [i + 1])), 0, i + 1)
            out += g * xt * nocc[:, i].reshape((ne,) + (1,) * K)
        return out.ravel()

    dim = int(np.prod(shape))
    op = spla.LinearOperator((dim, dim), matvec=matvec, dtype=float)
    rng = np.random.default_rng(0)
    w = spla.eigsh(op, k=1, which="SA", tol=1e-12, v0=rng.standard_normal(dim))[0]
    return float(w[0]), dim
