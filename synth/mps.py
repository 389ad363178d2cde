"""Seeded random MPS in block-sparse form (the paper's random initial guess).

A site tensor between bond k and bond k+1 is a dict {(il, s, ir): block} whose
block has shape (dim of sector il at bond k, dim of sector ir at bond k+1) and
exists when q(il) + q(s) = q(ir).

Right-canonical tensors have orthonormal rows over the fused (s, ir) index for
each left sector; left-canonical tensors have orthonormal columns over the fused
(il, s) index for each right sector.  Orthonormalising a Gaussian draw is how the
random guess is drawn; it is not part of the DMRG step being tested.
"""

import numpy as np

from .sectors import SITE_QN


def _index(bond):
    return {q: i for i, (q, _) in enumerate(bond)}


def _draw_right(rng, lbond, rbond):
    ridx = _index(rbond)
    t = {}
    for il, (ql, ml) in enumerate(lbond):
        cols = []
        for s, qs in enumerate(SITE_QN):
            qr = (ql[0] + qs[0], ql[1] + qs[1])
            if qr in ridx:
                cols.append((s, ridx[qr], rbond[ridx[qr]][1]))
        ncol = sum(c[2] for c in cols)
        if ncol < ml:
            raise ValueError("bond dims do not admit a right isometry")
        g = rng.standard_normal((ncol, ml))
        q, _ = np.linalg.qr(g)
        rows = q.T  # (ml, ncol), orthonormal rows
        off = 0
        for s, ir, mr in cols:
            t[(il, s, ir)] = np.ascontiguousarray(rows[:, off:off + mr])
            off += mr
    return t


def _draw_left(rng, lbond, rbond):
    lidx = _index(lbond)
    t = {}
    for ir, (qr, mr) in enumerate(rbond):
        rows = []
        for s, qs in enumerate(SITE_QN):
            ql = (qr[0] - qs[0], qr[1] - qs[1])
            if ql in lidx:
                rows.append((lidx[ql], s, lbond[lidx[ql]][1]))
        nrow = sum(r[2] for r in rows)
        if nrow < mr:
            raise ValueError("bond dims do not admit a left isometry")
        g = rng.standard_normal((nrow, mr))
        q, _ = np.linalg.qr(g)
        off = 0
        for il, s, ml in rows:
            t[(il, s, ir)] = np.ascontiguousarray(q[off:off + ml, :])
            off += ml
    return t


def random_right_canonical_mps(bonds, seed):
    """Site tensors 0..K-1, each right-canonical (bonds from bond_sector_tables)."""
    rng = np.random.default_rng(seed)
    K = len(bonds) - 1
    return [_draw_right(rng, bonds[k], bonds[k + 1]) for k in range(K)]


def random_left_canonical_mps(bonds, seed):
    """Site tensors 0..K-1, each left-canonical."""
    rng = np.random.default_rng(seed)
    K = len(bonds) - 1
    return [_draw_left(rng, bonds[k], bonds[k + 1]) for k in range(K)]
