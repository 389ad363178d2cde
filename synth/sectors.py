"""Quantum-number structure of the MPS bonds (U(1) x U(1): N and 2*Sz).

Site basis (Listing 1, electron part): [empty, alpha, beta, alpha-beta] with
quantum numbers (N, 2Sz) = (0,0), (1,1), (1,-1), (2,0).

A bond k (between site k-1 and site k) is labelled by the quantum number of the
*left* block (sites 0..k-1).  Bond 0 has the single sector (0,0) of dimension 1,
bond K the single sector (N, 2Sz) of the target state.

Sector dimensions for a random initial MPS (the paper's "random MPS with the
desired bond dimension"): every sector q that both blocks can hold gets a
capacity cap(q) = min(full left dim, full right dim) (the Schmidt-rank bound).
If the capacities sum to at most M the bond keeps them all (a complete basis);
otherwise M is shared in proportion to the number of full-space determinants
with that split, fl(q) * fr(q), capped at cap(q).  Dimensions are then trimmed so
that every site tensor can be an isometry from both sides.
"""

from math import comb

import numpy as np

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def site_shifts():
    """All (dN, d2Sz) a site operator can carry, with its (s_out, s_in) pairs."""
    out = {}
    for so, qo in enumerate(SITE_QN):
        for si, qi in enumerate(SITE_QN):
            d = (qo[0] - qi[0], qo[1] - qi[1])
            out.setdefault(d, []).append((so, si))
    return out


def _na_nb(q):
    n, tsz = q
    return (n + tsz) // 2, (n - tsz) // 2


def _full_dims(K, N, twosz, k):
    na_t, nb_t = (N + twosz) // 2, (N - twosz) // 2
    res = {}
    for na in range(0, k + 1):
        for nb in range(0, k + 1):
            fl = comb(k, na) * comb(k, nb)
            ra, rb = na_t - na, nb_t - nb
            if ra < 0 or rb < 0 or ra > K - k or rb > K - k:
                continue
            fr = comb(K - k, ra) * comb(K - k, rb)
            if fl > 0 and fr > 0:
                res[(na + nb, na - nb)] = (fl, fr)
    return res


def _distribute(full, M):
    caps = {q: min(fl, fr) for q, (fl, fr) in full.items()}
    if sum(caps.values()) <= M:
        return dict(caps)
    w = {q: float(fl) * float(fr) for q, (fl, fr) in full.items()}
    wsum = sum(w.values())

    def alloc(lam):
        return {q: min(caps[q], int(round(lam * M * w[q] / wsum))) for q in caps}

    lo, hi = 0.0, 1.0
    while sum(alloc(hi).values()) < M and hi < 1e30:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(alloc(mid).values()) <= M:
            lo = mid
        else:
            hi = mid
    return alloc(lo)


def _distribute_gaussian(full, M, k, K, N, twosz, width):
    na_t, nb_t = (N + twosz) / 2.0, (N - twosz) / 2.0
    caps = {q: min(fl, fr) for q, (fl, fr) in full.items()}
    w = {}
    for q in caps:
        na, nb = _na_nb(q)
        da, db = na - na_t * k / K, nb - nb_t * k / K
        w[q] = np.exp(-(da * da + db * db) / (2.0 * width * width))
    wsum = sum(w.values())

    def alloc(lam):
        return {q: min(caps[q], int(round(lam * M * w[q] / wsum))) for q in caps}

    if sum(caps.values()) <= M:
        return dict(caps)
    lo, hi = 0.0, 1.0
    while sum(alloc(hi).values()) < M and hi < 1e30:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(alloc(mid).values()) <= M:
            lo = mid
        else:
            hi = mid
    return alloc(lo)


def bond_sector_tables(K, N, twosz, M, model="proportional", width=1.0):
    """Return a list of K+1 bonds; each bond is a sorted list of ((N, 2Sz), dim).

    model="proportional": dims follow the determinant count of each split (the
    random initial MPS).  model="gaussian": dims follow
    exp(-(dNa^2 + dNb^2) / (2 width^2)), dNa/dNb the deviation of the left block's
    alpha/beta count from proportional filling; this mimics the concentrated
    sector distribution of a converged ground state.
    """
    dims = []
    for k in range(K + 1):
        full = _full_dims(K, N, twosz, k)
        if model == "gaussian":
            dims.append(_distribute_gaussian(full, M, k, K, N, twosz, width))
        else:
            dims.append(_distribute(full, M))
    dims[0] = {(0, 0): 1}
    dims[K] = {(N, twosz): 1}
    # trim so that left- and right-isometries exist at every site
    for _ in range(4 * K + 8):
        changed = False
        for k in range(K):  # forward: dim_{k+1}(q) <= sum_s dim_k(q - q_s)
            for q in list(dims[k + 1]):
                cap = sum(dims[k].get((q[0] - s[0], q[1] - s[1]), 0) for s in SITE_QN)
                if dims[k + 1][q] > cap:
                    dims[k + 1][q] = cap
                    changed = True
        for k in range(K - 1, -1, -1):  # backward: dim_k(q) <= sum_s dim_{k+1}(q + q_s)
            for q in list(dims[k]):
                cap = sum(dims[k + 1].get((q[0] + s[0], q[1] + s[1]), 0) for s in SITE_QN)
                if dims[k][q] > cap:
                    dims[k][q] = cap
                    changed = True
        if not changed:
            break
    return [sorted((q, m) for q, m in d.items() if m > 0) for d in dims]


def bond_stats(bond):
    ms = np.array([m for _, m in bond])
    return {"nsec": len(ms), "total": int(ms.sum()), "max": int(ms.max()), "min": int(ms.min())}
