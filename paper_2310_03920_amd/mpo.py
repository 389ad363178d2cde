"""Normal/complementary (NC) partition MPO for the ab initio Hamiltonian, with an
optional switch to the CN partition.

Sec. II.C.1 builds the ab initio Hamiltonian as a symbolic MPO whose bond
operators are the normal and complementary renormalised operators of
traditional DMRG, in the NC partition.  This module builds that MPO explicitly:

* Spin orbitals j = 2p + sigma, site-major (0a, 0b, 1a, 1b, ...).
* Site basis [empty, alpha, beta, alpha-beta] and on-site matrices c, d, C, D as
  printed in Listing 1; P = diag(1, -1, -1, 1) is the site parity.
* Bond operators at cut k (left block = sites 0..k-1), in the NC partition:
    I, H_L,
    C_x = a+_x, D_x = a_x                 (x in the left block),
    A_xy = a+_x a+_y, Ad_xy = a_y a_x     (x < y in the left block),
    B_xy = a+_x a_y                       (x, y in the left block),
    T_j, Td_j                             (j in the right block): the left-block
        factors of all terms whose only right-block operator is a_j (resp. a+_j),
        i.e. the left complementary operators of the single operators.
  Their right-block partners (H_R, the three-operator S terms, the pair
  operators P and Q, a_j / a+_j) are implied by the MPO recursion.
* Jordan-Wigner strings are carried by the MPO: the bond operator of an odd
  left-block operator X is X_JW times the left-block parity.  With this choice a
  bond operator at cut k+1 built from a bond operator at cut k and an on-site
  product x of ladder operators has site factor x . P^{parity of the new operator},
  and H = W^(0) W^(1) ... W^(K-1) with every product a plain Kronecker product.

* CN cuts (right of the switch cut of `build_mpo`, Sec. II.B.2): the same
  operators except that the left normal pairs A, Ad, B are replaced by the
  complementary pairs Pa_rs, Pd_rs, Q_rs (r, s right of the cut): the left
  factors, integrals included, of all two-body terms whose right part is
  a+_r a+_s, a_s a_r or a+_r a_s.  The bond then grows with the orbitals on the
  right, which is the smaller side past the middle of the chain.

Two-body coefficients: H2 = 1/2 sum V_ijkl a+_i a+_j a_k a_l with
V_ijkl = g[p_i, p_l, p_j, p_k] delta(s_i, s_l) delta(s_j, s_k) (chemists'
notation (pq|rs)); the one-body part is t_ij = h[p_i, p_j] delta(s_i, s_j).
"""

import itertools
from dataclasses import dataclass, field

import numpy as np

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))

_c = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]], float)
_d = _c.T.copy()
_C = np.array([[0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [0, -1, 0, 0]], float)
_D = _C.T.copy()
_P = np.diag([1.0, -1.0, -1.0, 1.0])
_I = np.eye(4)
CR = (_c, _C)  # a+_alpha, a+_beta
AN = (_d, _D)  # a_alpha, a_beta


def _spin_sign(j):
    return 1 if j % 2 == 0 else -1


def op_dq(key):
    """(dN, d2Sz) of a bond operator (as an operator on the left block)."""
    kind = key[0]
    if kind in ("I", "H"):
        return (0, 0)
    if kind == "C":
        return (1, _spin_sign(key[1]))
    if kind == "D":
        return (-1, -_spin_sign(key[1]))
    if kind == "A":
        return (2, _spin_sign(key[1]) + _spin_sign(key[2]))
    if kind == "Ad":
        return (-2, -_spin_sign(key[1]) - _spin_sign(key[2]))
    if kind == "B":
        return (0, _spin_sign(key[1]) - _spin_sign(key[2]))
    if kind == "T":   # partner of a_j: left factor carries +dq(a+_j)
        return (1, _spin_sign(key[1]))
    if kind == "Td":
        return (-1, -_spin_sign(key[1]))
    # complementary pair operators: minus the change of their right partner
    if kind == "Pa":  # partner a+_r a+_s
        return (-2, -_spin_sign(key[1]) - _spin_sign(key[2]))
    if kind == "Pd":  # partner a_s a_r
        return (2, _spin_sign(key[1]) + _spin_sign(key[2]))
    if kind == "Q":   # partner a+_r a_s
        return (0, _spin_sign(key[2]) - _spin_sign(key[1]))
    raise KeyError(key)


def op_parity(key):
    return 1 if key[0] in ("C", "D", "T", "Td") else 0


def cut_ops(K, k, cn=False):
    """Bond operators at cut k (before pruning), in a fixed order.

    NC cut: normal pair operators A, Ad, B of the left block.  CN cut: in their
    place the complementary pair operators Pa_rs, Pd_rs, Q_rs (r, s right of the
    cut), each the left factor of all two-body terms whose right part is
    a+_r a+_s, a_s a_r or a+_r a_s respectively (r < s for Pa and Pd)."""
    ops = []
    if k < K:
        ops.append(("I",))
    if k >= 1:
        ops.append(("H",))
    if 0 < k < K:
        n = 2 * k
        ops += [("C", x) for x in range(n)]
        ops += [("D", x) for x in range(n)]
        if not cn:
            ops += [("A", x, y) for x in range(n) for y in range(x + 1, n)]
            ops += [("Ad", x, y) for x in range(n) for y in range(x + 1, n)]
            ops += [("B", x, y) for x in range(n) for y in range(n)]
        ops += [("T", j) for j in range(n, 2 * K)]
        ops += [("Td", j) for j in range(n, 2 * K)]
        if cn:
            m = range(n, 2 * K)
            ops += [("Pa", r, s) for r in m for s in m if r < s]
            ops += [("Pd", r, s) for r in m for s in m if r < s]
            ops += [("Q", r, s) for r in m for s in m]
    return ops


class _Coef:
    """Spin-orbital one- and two-body coefficients from spatial integrals."""

    def __init__(self, h, g):
        self.h, self.g = h, g

    def t(self, i, j):
        i, j = np.asarray(i), np.asarray(j)
        return self.h[i // 2, j // 2] * ((i % 2) == (j % 2))

    def v(self, i, j, k, l):
        i, j, k, l = (np.asarray(x) for x in (i, j, k, l))
        return (self.g[i // 2, l // 2, j // 2, k // 2]
                * ((i % 2) == (l % 2)) * ((j % 2) == (k % 2)))


def _inversions(regions):
    inv = 0
    for p in range(len(regions)):
        for q in range(p + 1, len(regions)):
            if regions[p] > regions[q]:
                inv += 1
    return inv


@dataclass
class SiteMPO:
    """W^(k): entries (row op index at cut k, column op index at cut k+1, 4x4)."""
    rows: np.ndarray
    cols: np.ndarray
    mats: np.ndarray


@dataclass
class MPO:
    K: int
    cuts: list            # cuts[k] = list of op keys at cut k (after pruning)
    sites: list           # sites[k] = SiteMPO between cut k and cut k+1
    dq: list = field(default_factory=list)      # dq[k] = (n_ops, 2) int array
    parity: list = field(default_factory=list)  # parity[k] = (n_ops,) int array


class _Index:
    """Vectorised lookup from operator keys to positions in a cut's operator list."""

    def __init__(self, K, ops):
        n2 = 2 * K
        self.I = self.H = -1
        self.C = np.full(n2, -1)
        self.D = np.full(n2, -1)
        self.A = np.full((n2, n2), -1)
        self.Ad = np.full((n2, n2), -1)
        self.B = np.full((n2, n2), -1)
        self.T = np.full(n2, -1)
        self.Td = np.full(n2, -1)
        self.Pa = np.full((n2, n2), -1)
        self.Pd = np.full((n2, n2), -1)
        self.Q = np.full((n2, n2), -1)
        for i, key in enumerate(ops):
            kind = key[0]
            if kind == "I":
                self.I = i
            elif kind == "H":
                self.H = i
            elif kind in ("C", "D", "T", "Td"):
                getattr(self, kind)[key[1]] = i
            else:
                getattr(self, kind)[key[1], key[2]] = i


class _Sink:
    """Collects (row, col, coef, site matrix) in arrays; sums duplicates at the end."""

    def __init__(self):
        self.rows, self.cols, self.mats = [], [], []

    def add(self, rows, cols, coef, site):
        rows = np.atleast_1d(np.asarray(rows)).ravel()
        cols = np.broadcast_to(np.atleast_1d(np.asarray(cols)).ravel(), rows.shape)
        coef = np.broadcast_to(np.atleast_1d(np.asarray(coef, float)).ravel(), rows.shape)
        keep = (rows >= 0) & (cols >= 0) & (coef != 0.0)
        if not np.any(keep):
            return
        self.rows.append(rows[keep])
        self.cols.append(cols[keep])
        self.mats.append(coef[keep][:, None, None] * site[None, :, :])

    def result(self):
        if not self.rows:
            return np.zeros(0, int), np.zeros(0, int), np.zeros((0, 4, 4))
        r = np.concatenate(self.rows)
        c = np.concatenate(self.cols)
        m = np.concatenate(self.mats)
        order = np.lexsort((r, c))
        r, c, m = r[order], c[order], m[order]
        first = np.ones(len(r), bool)
        first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
        starts = np.nonzero(first)[0]
        return r[starts], c[starts], np.add.reduceat(m, starts, axis=0)


def _site_entries(K, k, coef, ops_k, ops_k1, rows_cn=False, cols_cn=False):
    """W^(k) entries as arrays (row op index at cut k, col op index at cut k+1, 4x4).

    rows_cn / cols_cn: cut k / cut k+1 is a CN cut (complementary pair operators
    instead of normal ones).  NC rows with CN columns is the switch site, where
    the integrals are folded into the left normal pairs."""
    ik, ik1 = _Index(K, ops_k), _Index(K, ops_k1)
    out = _Sink()
    n = 2 * k
    kap = (2 * k, 2 * k + 1)
    xs = np.arange(n)
    # identity propagation and normal operators
    out.add(ik.I, ik1.I, 1.0, _I)
    out.add(ik.H, ik1.H, 1.0, _I)
    out.add(ik.C[xs], ik1.C[xs], 1.0, _P)
    out.add(ik.D[xs], ik1.D[xs], 1.0, _P)
    for s in range(2):
        out.add(ik.I, ik1.C[kap[s]], 1.0, CR[s] @ _P)
        out.add(ik.I, ik1.D[kap[s]], 1.0, AN[s] @ _P)
    if not cols_cn:
        if n:
            X, Y = np.meshgrid(xs, xs, indexing="ij")
            up = X < Y
            out.add(ik.A[X[up], Y[up]], ik1.A[X[up], Y[up]], 1.0, _I)
            out.add(ik.Ad[X[up], Y[up]], ik1.Ad[X[up], Y[up]], 1.0, _I)
            out.add(ik.B[X, Y], ik1.B[X, Y], 1.0, _I)
        for s in range(2):
            out.add(ik.C[xs], ik1.A[xs, kap[s]], 1.0, CR[s])
            out.add(ik.D[xs], ik1.Ad[xs, kap[s]], -1.0, AN[s])
            out.add(ik.C[xs], ik1.B[xs, kap[s]], 1.0, AN[s])
            out.add(ik.D[xs], ik1.B[kap[s], xs], -1.0, CR[s])
        out.add(ik.I, ik1.A[kap[0], kap[1]], 1.0, CR[0] @ CR[1])
        out.add(ik.I, ik1.Ad[kap[0], kap[1]], 1.0, AN[1] @ AN[0])
        for s in range(2):
            for t in range(2):
                out.add(ik.I, ik1.B[kap[s], kap[t]], 1.0, CR[s] @ AN[t])
    js = np.arange(2 * k + 2, 2 * K)
    out.add(ik.T[js], ik1.T[js], 1.0, _P)
    out.add(ik.Td[js], ik1.Td[js], 1.0, _P)
    # H picks up the complementary operators of the new site's single operators
    for s in range(2):
        out.add(ik.T[kap[s]], ik1.H, 1.0, AN[s])
        out.add(ik.Td[kap[s]], ik1.H, 1.0, CR[s])
    if rows_cn:
        # Complementary pairs of a CN cut already hold their integrals: pairs
        # right of site k carry on; a pair on site k closes into H (times the
        # partner on the site); a pair (site k, j) becomes part of T_j or Td_j.
        # Sum over terms = sum_O P_O * O, so with x the site factor and
        # O = eta * x * a_j (or a+_j), T_j (Td_j) gains eta * P_O (x) x . P.
        R, S = np.meshgrid(js, js, indexing="ij")
        up = R < S
        out.add(ik.Pa[R[up], S[up]], ik1.Pa[R[up], S[up]], 1.0, _I)
        out.add(ik.Pd[R[up], S[up]], ik1.Pd[R[up], S[up]], 1.0, _I)
        out.add(ik.Q[R, S], ik1.Q[R, S], 1.0, _I)
        out.add(ik.Pa[kap[0], kap[1]], ik1.H, 1.0, CR[0] @ CR[1])
        out.add(ik.Pd[kap[0], kap[1]], ik1.H, 1.0, AN[1] @ AN[0])
        for s in range(2):
            for t in range(2):
                out.add(ik.Q[kap[s], kap[t]], ik1.H, 1.0, CR[s] @ AN[t])
        for s in range(2):
            out.add(ik.Q[kap[s], js], ik1.T[js], 1.0, CR[s] @ _P)     # a+_ks a_j
            out.add(ik.Pd[kap[s], js], ik1.T[js], -1.0, AN[s] @ _P)   # a_j a_ks = -a_ks a_j
            out.add(ik.Pa[kap[s], js], ik1.Td[js], 1.0, CR[s] @ _P)   # a+_ks a+_j
            out.add(ik.Q[js, kap[s]], ik1.Td[js], -1.0, AN[s] @ _P)   # a+_j a_ks = -a_ks a+_j

    # remaining H and T/Td contributions: enumerate operator-slot patterns
    Lidx = xs
    outs = js
    one = ((True, False), lambda a, b: coef.t(a, b))
    two = ((True, True, False, False), lambda a, b, c, d: 0.5 * coef.v(a, b, c, d))

    def slot_patterns(nslot, target):
        # region per slot: 0 = left block, 1 = site k, 2 = outside operator
        for regs in itertools.product((0, 1, 2), repeat=nslot):
            nk = regs.count(1)
            nout = regs.count(2)
            if target == "H":
                if nout or nk < 2:
                    continue
            elif target == "P":
                # a left pair of a CN cut carries on by itself; at the switch
                # the left normal pair is contracted with the integrals here
                if nout != 2 or nslot != 4 or (nk == 0 and rows_cn):
                    continue
            elif nout != 1 or nk < 1:
                continue
            if rows_cn and target != "P" and regs.count(0) == 2:
                continue  # from the complementary pairs above
            yield regs

    targets = ("H", "T", "Td") + (("P",) if cols_cn else ())
    for daggers, cfn in (one, two):
        ns = len(daggers)
        for target in targets:
            if target != "H" and len(outs) == 0:
                continue
            for regs in slot_patterns(ns, target):
                if target in ("T", "Td"):
                    pos = regs.index(2)
                    if target == "T" and daggers[pos]:
                        continue
                    if target == "Td" and not daggers[pos]:
                        continue
                lslots = [p for p in range(ns) if regs[p] == 0]
                kslots = [p for p in range(ns) if regs[p] == 1]
                if len(lslots) > 2 or (lslots and n == 0):
                    continue
                sign = -1.0 if _inversions(regs) % 2 else 1.0
                par_b = 1 if target in ("T", "Td") else 0
                for spins in itertools.product(range(2), repeat=len(kslots)):
                    site = _I
                    for p, s in zip(kslots, spins):
                        site = site @ (CR[s] if daggers[p] else AN[s])
                    if not np.any(site):
                        continue
                    if par_b:
                        site = site @ _P
                    grids = []
                    for p in range(ns):
                        if regs[p] == 0:
                            grids.append(Lidx)
                        elif regs[p] == 1:
                            grids.append(np.array([kap[spins[kslots.index(p)]]]))
                        else:
                            grids.append(outs)
                    mesh = np.meshgrid(*grids, indexing="ij")
                    cval = sign * cfn(*mesh)
                    keep_axes = [p for p in range(ns) if regs[p] != 1]
                    cval = cval.reshape([len(grids[p]) for p in keep_axes])
                    _emit(out, ik, ik1, target, daggers, lslots, regs, cval, site, outs)
    return out.result()


def _emit(out, ik, ik1, target, daggers, lslots, regs, cval, site, outs):
    """Distribute a coefficient array onto canonical left operators (vectorised)."""
    ld = [daggers[p] for p in lslots]
    kept = [p for p in range(len(regs)) if regs[p] != 1]
    if target == "H":
        cval = cval[..., None]
        cols = np.array([ik1.H])
    elif target == "P":
        # outside pair (slot order) -> canonical complementary pair and its sign
        o1, o2 = [p for p in range(len(regs)) if regs[p] == 2]
        cval = np.moveaxis(cval, [kept.index(o1), kept.index(o2)], [-2, -1])
        R, S = np.meshgrid(outs, outs, indexing="ij")
        lo, hi = np.minimum(R, S), np.maximum(R, S)
        if daggers[o1] and daggers[o2]:      # a+_r a+_s = +-Pa partner
            cols, sg = ik1.Pa[lo, hi], np.sign(S - R)
        elif not daggers[o1] and not daggers[o2]:  # a_r a_s: partner a_hi a_lo
            cols, sg = ik1.Pd[lo, hi], np.sign(R - S)
        else:                                # a+_r a_s
            cols, sg = ik1.Q[R, S], np.ones_like(R)
        cval = (cval * sg).reshape(cval.shape[:-2] + (-1,))
        cols = cols.ravel()
    else:
        oax = kept.index(regs.index(2))
        cval = np.moveaxis(cval, oax, -1)  # outside index last
        cols = (ik1.T if target == "T" else ik1.Td)[outs]
    nj = len(cols)
    if len(lslots) == 0:
        out.add(np.full(nj, ik.I), cols, cval.reshape(nj), site)
    elif len(lslots) == 1:
        idx = ik.C if ld[0] else ik.D
        nl = cval.shape[0]
        rows = np.repeat(idx[:nl], nj)
        out.add(rows, np.tile(cols, nl), cval.reshape(nl * nj), site)
    else:
        nl = cval.shape[0]
        X, Y = np.meshgrid(np.arange(nl), np.arange(nl), indexing="ij")
        up = X < Y
        if ld == [True, True]:      # a+_x a+_y = A_xy (x<y), -A_yx (x>y)
            m = cval - np.swapaxes(cval, 0, 1)
            rows = ik.A[X[up], Y[up]]
        elif ld == [False, False]:  # a_x a_y = Ad_yx (y<x), -Ad_xy (x<y); Ad_jl = a_l a_j
            m = np.swapaxes(cval, 0, 1) - cval
            rows = ik.Ad[X[up], Y[up]]
        elif ld == [True, False]:   # a+_x a_y = B_xy
            m = cval
            up = np.ones_like(up)
            rows = ik.B[X[up], Y[up]]
        else:
            raise AssertionError("left factor not normal ordered")
        vals = m[X[up], Y[up]]                       # (npair, nj)
        out.add(np.repeat(rows, nj), np.tile(cols, len(rows)), vals.reshape(-1), site)


def build_nc_mpo(h, g, prune=True, tol=0.0):
    """Return the NC-partition MPO of H(h, g) for K = h.shape[0] orbitals."""
    return build_mpo(h, g, switch=None, prune=prune, tol=tol)


def build_mpo(h, g, switch=None, prune=True, tol=0.0):
    """MPO of H(h, g) in the NC partition up to cut `switch` and the CN partition
    after it (Sec. II.B.2: normal operators on the smaller side of each cut).
    switch=None is NC everywhere; switch=K//2 keeps every bond near 8 k^2 with k
    the orbitals on the smaller side instead of the left one.  The operator is the
    same for every switch position; only the bond operators differ."""
    K = h.shape[0]
    sw = K if switch is None else int(switch)
    if not 0 <= sw <= K:
        raise ValueError(f"switch cut must be in 0 .. {K}")
    coef = _Coef(np.asarray(h, float), np.asarray(g, float))
    cuts = [cut_ops(K, k, cn=k > sw) for k in range(K + 1)]
    raw = []
    for k in range(K):
        r, c, m = _site_entries(K, k, coef, cuts[k], cuts[k + 1], rows_cn=k > sw, cols_cn=k + 1 > sw)
        keep = np.abs(m).reshape(len(m), -1).max(axis=1) > tol if len(m) else np.zeros(0, bool)
        raw.append((r[keep], c[keep], m[keep]))
    alive = [np.ones(len(c), bool) for c in cuts]
    if prune:
        changed = True
        while changed:
            changed = False
            for k in range(K):
                used_in = np.zeros(len(cuts[k + 1]), bool)
                used_out = np.zeros(len(cuts[k]), bool)
                ra, rb, _ = raw[k]
                both = alive[k][ra] & alive[k + 1][rb]
                used_in[rb[both]] = True
                used_out[ra[both]] = True
                new1 = alive[k + 1] & used_in
                new0 = alive[k] & used_out
                if (new1 != alive[k + 1]).any() or (new0 != alive[k]).any():
                    changed = True
                alive[k + 1], alive[k] = new1, new0
    remap = []
    new_cuts = []
    for k in range(K + 1):
        m = -np.ones(len(cuts[k]), int)
        keep = np.nonzero(alive[k])[0]
        m[keep] = np.arange(len(keep))
        remap.append(m)
        new_cuts.append([cuts[k][i] for i in keep])
    sites = []
    for k in range(K):
        ra, rb, mats = raw[k]
        na, nb = remap[k][ra], remap[k + 1][rb]
        ok = (na >= 0) & (nb >= 0)
        na, nb, mats = na[ok], nb[ok], mats[ok]
        order = np.lexsort((na, nb))
        sites.append(SiteMPO(na[order].astype(np.int32), nb[order].astype(np.int32), mats[order]))
    mpo = MPO(K, new_cuts, sites)
    mpo.dq = [np.array([op_dq(key) for key in c], np.int32).reshape(-1, 2) for c in new_cuts]
    mpo.parity = [np.array([op_parity(key) for key in c], np.int32) for c in new_cuts]
    return mpo


def site_entries(mpo, k):
    """W^(k) as a list of (row, col, 4x4) for the block formats used in tests."""
    s = mpo.sites[k]
    return [(int(a), int(b), m) for a, b, m in zip(s.rows, s.cols, s.mats)]


def densify(mpo):
    """Contract the whole MPO to a dense 4^K x 4^K matrix (small K only)."""
    cur = np.ones((1, 1, 1))  # (op at cut 0, bra, ket)
    for k in range(mpo.K):
        s = mpo.sites[k]
        D1 = len(mpo.cuts[k + 1])
        n = cur.shape[1]
        nxt = np.zeros((D1, n * 4, n * 4))
        for a, b, m in zip(s.rows, s.cols, s.mats):
            nxt[b] += np.kron(cur[a], m)
        cur = nxt
    assert cur.shape[0] == 1
    return cur[0]
