"""Seeded random block-sparse operands for kernel-level tests and benchmarks.

Formats (shared vocabulary of both sides; plain dicts of numpy arrays):

* bond: sorted list of ((N, 2Sz), dim).
* two-site wavefunction between bond i and bond i+2: {(il, s1, s2, ir): block}
  with block shape (dim il, dim ir), present when q(il)+q(s1)+q(s2) = q(ir).
* environment: list of operators, each {"dq": (dN, d2Sz), "blocks": {isrc: blk}}
  where blk has shape (dim of sector q(isrc)+dq, dim of isrc).  Left and right
  environments use the same convention on their own bond's sector labels.
* MPO site entries: list of (row, col, op) with op a dense 4x4 matrix over the
  site basis [empty, alpha, beta, alpha-beta]; op shifts the site quantum number
  by dq(col) - dq(row).
"""

import numpy as np

from .sectors import SITE_QN, site_shifts


def _index(bond):
    return {q: i for i, (q, _) in enumerate(bond)}


def _add(q, d):
    return (q[0] + d[0], q[1] + d[1])


def two_site_blocks(lbond, rbond):
    ridx = _index(rbond)
    keys = []
    for il, (ql, _) in enumerate(lbond):
        for s1, q1 in enumerate(SITE_QN):
            for s2, q2 in enumerate(SITE_QN):
                qr = _add(_add(ql, q1), q2)
                if qr in ridx:
                    keys.append((il, s1, s2, ridx[qr]))
    return keys


def random_psi(lbond, rbond, rng):
    out = {}
    for key in two_site_blocks(lbond, rbond):
        il, _, _, ir = key
        out[key] = rng.standard_normal((lbond[il][1], rbond[ir][1]))
    return out


def random_env(bond, dqs, rng, scale=1.0):
    idx = _index(bond)
    ops = []
    for dq in dqs:
        blocks = {}
        for isrc, (q, m) in enumerate(bond):
            qd = _add(q, dq)
            if qd in idx:
                blocks[isrc] = scale * rng.standard_normal((bond[idx[qd]][1], m))
        ops.append({"dq": tuple(dq), "blocks": blocks})
    return ops


def random_site_ops(dq_rows, dq_cols, rng, per_col=3, identity_frac=0.3):
    """Random MPO entries (row, col, op) with quantum-number-consistent shifts."""
    shifts = site_shifts()
    rows_by_dq = {}
    for a, d in enumerate(dq_rows):
        rows_by_dq.setdefault(tuple(d), []).append(a)
    entries = []
    for b, db in enumerate(dq_cols):
        cand = []
        for dsite in shifts:
            da = (db[0] - dsite[0], db[1] - dsite[1])
            for a in rows_by_dq.get(da, []):
                cand.append((a, dsite))
        if not cand:
            continue
        pick = rng.choice(len(cand), size=min(per_col, len(cand)), replace=False)
        for p in sorted(pick):
            a, dsite = cand[p]
            op = np.zeros((4, 4))
            for so, si in shifts[dsite]:
                if dsite == (0, 0) and rng.random() < identity_frac:
                    op[so, si] = 1.0
                else:
                    op[so, si] = rng.standard_normal()
            entries.append((a, b, op))
    return entries


def random_site_tensor(lbond, rbond, rng):
    """Unconstrained random site tensor {(il, s, ir): block}."""
    ridx = _index(rbond)
    t = {}
    for il, (ql, ml) in enumerate(lbond):
        for s, qs in enumerate(SITE_QN):
            qr = _add(ql, qs)
            if qr in ridx:
                t[(il, s, ridx[qr])] = rng.standard_normal((ml, rbond[ridx[qr]][1]))
    return t
