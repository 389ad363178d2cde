"""Fock-space definition of the ab initio Hamiltonian (Sec. II.A.1).

Spin-orbital j = 2p + sigma (sigma = 0 alpha, 1 beta), i.e. the site-major
ordering 0a, 0b, 1a, 1b, ...  An occupation bit string `occ` stands for the
determinant prod_{j ascending} (a_j^dagger)^{n_j} |vac>.  With this ordering a
spatial orbital's doubly occupied state is a_alpha^dagger a_beta^dagger |0>,
which is the sign convention of the on-site matrices printed in Listing 1.

H = sum_pq h_pq sum_s a+_ps a_qs + 1/2 sum_pqrs g_pqrs sum_st a+_ps a+_rt a_st a_qs
  (chemists' notation (pq|rs), core energy zero), equivalently
H = sum_pq (h_pq - 1/2 sum_r g_prrq) E_pq + 1/2 sum_pqrs g_pqrs E_pq E_rs with
E_pq = sum_s a+_ps a_qs.
"""

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


def apply_op(occ, j, dagger):
    """Apply a_j^dagger (dagger=True) or a_j to determinants `occ` (int array).

    Returns (sign, new_occ); sign is 0 where the result vanishes.
    """
    occ = np.asarray(occ, dtype=np.int64)
    bit = np.int64(1) << np.int64(j)
    occupied = (occ & bit) != 0
    sign = np.where(popcount(occ & (bit - 1)) % 2 == 0, 1.0, -1.0)
    if dagger:
        ok = ~occupied
        new = occ | bit
    else:
        ok = occupied
        new = occ & ~bit
    return np.where(ok, sign, 0.0), np.where(ok, new, occ)


def sector_dets(K, N, twosz):
    """Sorted determinants of K spatial orbitals with N electrons and 2Sz = twosz."""
    na, nb = (N + twosz) // 2, (N - twosz) // 2
    if na < 0 or nb < 0 or na > K or nb > K or na + nb != N:
        return np.zeros(0, dtype=np.int64)
    dets = []
    for a in itertools.combinations(range(K), na):
        for b in itertools.combinations(range(K), nb):
            occ = 0
            for p in a:
                occ |= 1 << (2 * p)
            for p in b:
                occ |= 1 << (2 * p + 1)
            dets.append(occ)
    return np.array(sorted(dets), dtype=np.int64)


def all_dets(K):
    return np.arange(1 << (2 * K), dtype=np.int64)


def op_matrix(dets, ops):
    """Sparse matrix of a product of ladder operators on the span of `dets`.

    ops: list of (j, dagger) applied right-to-left as written left-to-right, i.e.
    ops = [(i, True), (j, False)] is a+_i a_j.  Results leaving the span are
    dropped (callers only use sector-preserving products).
    """
    dets = np.asarray(dets, dtype=np.int64)
    sign = np.ones(len(dets))
    cur = dets.copy()
    for j, dag in reversed(ops):
        s, cur = apply_op(cur, j, dag)
        sign = sign * s
    pos = np.searchsorted(dets, cur)
    pos = np.clip(pos, 0, len(dets) - 1)
    inside = (dets[pos] == cur) & (sign != 0)
    cols = np.nonzero(inside)[0]
    return sp.csr_matrix((sign[inside], (pos[inside], cols)), shape=(len(dets), len(dets)))


def excitation_ops(dets, K):
    """E_pq = sum_sigma a+_{p sigma} a_{q sigma} on the span of `dets`."""
    E = {}
    for p in range(K):
        for q in range(K):
            E[(p, q)] = (op_matrix(dets, [(2 * p, True), (2 * q, False)])
                         + op_matrix(dets, [(2 * p + 1, True), (2 * q + 1, False)]))
    return E


def hamiltonian(h, g, dets):
    """H on the span of `dets` (sparse CSR), from the E_pq form in the header."""
    K = h.shape[0]
    n = len(dets)
    E = excitation_ops(dets, K)
    Ecoo = {k: v.tocoo() for k, v in E.items()}
    rows = np.concatenate([Ecoo[(r, s)].row for r in range(K) for s in range(K)])
    cols = np.concatenate([Ecoo[(r, s)].col for r in range(K) for s in range(K)])
    vals = np.concatenate([Ecoo[(r, s)].data for r in range(K) for s in range(K)])
    rs_of = np.concatenate([np.full(Ecoo[(r, s)].nnz, r * K + s) for r in range(K) for s in range(K)])
    tp = h - 0.5 * np.einsum("prrq->pq", g)
    one = tp.ravel()[rs_of] * vals
    H = sp.coo_matrix((one, (rows, cols)), shape=(n, n)).tocsr()
    for p in range(K):
        for q in range(K):
            coef = g[p, q].ravel()[rs_of] * vals
            if not np.any(coef):
                continue
            X = sp.coo_matrix((coef, (rows, cols)), shape=(n, n)).tocsr()
            H = H + 0.5 * (E[(p, q)] @ X)
    H.eliminate_zeros()
    return H.tocsr()


def hamiltonian_bruteforce(h, g, dets):
    """H assembled term by term from the second-quantised definition (tiny K)."""
    K = h.shape[0]
    n = len(dets)
    H = sp.csr_matrix((n, n))
    for p in range(K):
        for q in range(K):
            for s in range(2):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * op_matrix(dets, [(2 * p + s, True), (2 * q + s, False)])
    for p, q, r, s in itertools.product(range(K), repeat=4):
        if g[p, q, r, s] == 0.0:
            continue
        for si in range(2):
            for ti in range(2):
                H = H + 0.5 * g[p, q, r, s] * op_matrix(
                    dets, [(2 * p + si, True), (2 * r + ti, True), (2 * s + ti, False), (2 * q + si, False)])
    return H.tocsr()


def one_rdm(vec, dets, K):
    """Spin-summed 1-RDM gamma_pq = <v| E_pq |v> (Sec. II.E.1) of a real vector on
    the span of `dets`."""
    E = excitation_ops(dets, K)
    return np.array([[vec @ (E[(p, q)] @ vec) for q in range(K)] for p in range(K)])


def two_rdm(vec, dets, K):
    """Spin-summed 2-RDM Gamma_pqrs = <v| sum_st a+_ps a+_rt a_st a_qs |v> (Sec. II.E.1),
    from the anticommutation identity sum_st a+_ps a+_rt a_st a_qs = E_pq E_rs -
    delta_qr E_ps.  With it E = sum h_pq gamma_pq + 1/2 sum g_pqrs Gamma_pqrs for the
    Hamiltonian of this module."""
    E = excitation_ops(dets, K)
    Ev = {k: m @ vec for k, m in E.items()}
    G = np.zeros((K, K, K, K))
    for p in range(K):
        for q in range(K):
            left = E[(q, p)] @ vec  # <v| E_pq = (E_qp v)^T
            for r in range(K):
                for s in range(K):
                    G[p, q, r, s] = left @ Ev[(r, s)]
    gam = np.array([[vec @ Ev[(p, q)] for q in range(K)] for p in range(K)])
    for q in range(K):
        G[:, q, q, :] -= gam
    return G


def fci_energy(h, g, N, twosz, nroots=1):
    K = h.shape[0]
    dets = sector_dets(K, N, twosz)
    H = hamiltonian(h, g, dets)
    if len(dets) <= 2000:
        w = np.linalg.eigvalsh(H.toarray())
        return w[:nroots] if nroots > 1 else float(w[0])
    w = spla.eigsh(H, k=max(nroots, 1), which="SA", tol=1e-13, maxiter=100000)[0]
    w = np.sort(w)
    return w[:nroots] if nroots > 1 else float(w[0])


def product_index(dets, K):
    """Index of each determinant in the site-product basis (s_0 most significant).

    Site state s_p = n_{p alpha} + 2 n_{p beta}, i.e. [empty, alpha, beta, alpha-beta].
    """
    dets = np.asarray(dets, dtype=np.int64)
    idx = np.zeros(len(dets), dtype=np.int64)
    for p in range(K):
        s = ((dets >> (2 * p)) & 1) + 2 * ((dets >> (2 * p + 1)) & 1)
        idx = idx * 4 + s
    return idx
