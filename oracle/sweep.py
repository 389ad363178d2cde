"""Two-site DMRG sweep with truncation, by definition (Sec. II.A.2).

TEST INFRASTRUCTURE ONLY (see the package docstring): no product code calls this
module, and it shares no code with the HIP library or its Python binding.

The sweep the paper describes optimises two neighbouring sites at a time, splits
the optimised two-site tensor with a singular value decomposition that keeps the
M largest singular values (the bond dimension), and moves one site on; passes
alternate in direction.  Each site step here is:

  1. the two-site tensor psi0 = (centre) x (neighbour) of the current MPS;
  2. the lowest eigenpair of the two-site effective Hamiltonian over the blocks
     the symmetry allows, by a library eigensolver (dense `eigh` for small
     spaces, ARPACK `eigsh` otherwise; psi0 is only a start vector);
  3. the split: psi is a block-diagonal matrix between (left bond, site 1) and
     (site 2, right bond), one block per quantum number Q of the new middle bond.
     Each block gets a FULL SVD (the square factor on the side being kept, whose
     null-space columns carry singular value 0).  Over all blocks the M largest
     singular values are kept, zeros included when fewer than M are non-zero;
     the discarded weight is the sum of the dropped s^2;
  4. the kept left (or right) singular vectors become the new canonical site
     tensor, S V^T (or U S) the centre carried to the next step.

Readings where the paper is silent (the same ones the product takes):
  * passes alternate, the first left to right over the pairs (0,1)..(K-2,K-1);
    the end pair of a pass is split towards the next pass, which starts one pair
    in (so a pass after the first has K-2 steps);
  * sector order is lexicographic (N, 2Sz); equal singular values are ordered by
    (sector, index within the sector), where values within TIE_RTOL * s_max of
    the first value of a run of near-equal values count as equal -- the spin
    multiplets of a spin-free Hamiltonian give exactly equal singular values in
    different 2Sz sectors, which rounding would otherwise order at random.

Two effective Hamiltonians are provided, both plain definitions:
  * FockHeff: H_eff := P^T H P with P the isometry of the MPS basis into Fock space
    (oracle.mps), H the Fock-space Hamiltonian (oracle.fock): no MPO and no
    environments (small chains only);
  * MpoHeff: the renormalised-operator contraction of oracle.contract on dense
    zero-padded environments, which are built from scratch at every step from the
    MPS tensors; the MPO values are passed in as data.
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import contract, fock
from . import mps as omps

SITE_Q = ((0, 0), (1, 1), (1, -1), (2, 0))   # (N, 2Sz) of [empty, alpha, beta, alpha-beta]
TIE_RTOL = 1e-8


def _qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


# ------------------------------------------------------------------ step 1: the two-site tensor

def merge(left, right, lbond, mbond, rbond):
    """theta[(il, s1, s2, ir)] = sum_m left[(il, s1, m)] @ right[(m, s2, ir)]."""
    out = {}
    for (il, s1, m), a in left.items():
        for (m2, s2, ir), b in right.items():
            if m2 != m:
                continue
            key = (il, s1, s2, ir)
            out[key] = out.get(key, 0.0) + a @ b
    return out


def allowed_blocks(lbond, rbond):
    """Two-site blocks (il, s1, s2, ir) with q(il)+q(s1)+q(s2) = q(ir)."""
    ridx = {q: j for j, (q, _) in enumerate(rbond)}
    keys = []
    for il, (ql, _) in enumerate(lbond):
        for s1 in range(4):
            for s2 in range(4):
                q = _qadd(_qadd(ql, SITE_Q[s1]), SITE_Q[s2])
                if q in ridx:
                    keys.append((il, s1, s2, ridx[q]))
    return keys


def to_vector(psi, lbond, rbond, keys):
    parts = []
    for k in keys:
        il, _, _, ir = k
        blk = psi.get(k)
        parts.append(np.zeros(lbond[il][1] * rbond[ir][1]) if blk is None else np.asarray(blk).ravel())
    return np.concatenate(parts) if parts else np.zeros(0)


def from_vector(vec, lbond, rbond, keys):
    out, o = {}, 0
    for k in keys:
        il, _, _, ir = k
        n = lbond[il][1] * rbond[ir][1]
        out[k] = vec[o:o + n].reshape(lbond[il][1], rbond[ir][1]).copy()
        o += n
    return out


# ------------------------------------------------------------------ step 2: the eigenproblem

def lowest_eigenpair(matvec, n, v0, dense_max=600):
    """Lowest eigenpair of a symmetric operator of size n given by `matvec`
    (library eigensolvers; no Davidson code)."""
    if n <= dense_max:
        H = np.column_stack([matvec(e) for e in np.eye(n)]) if n else np.zeros((0, 0))
        H = 0.5 * (H + H.T)
        w, U = np.linalg.eigh(H)
        return float(w[0]), U[:, 0]
    op = spla.LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    start = v0 if v0 is not None and np.linalg.norm(v0) > 0 else None
    w, U = spla.eigsh(op, k=1, which="SA", v0=start, tol=0.0, ncv=min(n - 1, 48), maxiter=100000)
    return float(w[0]), U[:, 0]


class FockHeff:
    """H_eff := P^T H P for the two-site step at (i, i+1); P from the MPS tensors
    left of i (left-canonical) and right of i+1 (right-canonical)."""

    def __init__(self, h, g, n_elec, twosz):
        self.K = h.shape[0]
        self.dets = fock.sector_dets(self.K, n_elec, twosz)
        self.pidx = fock.product_index(self.dets, self.K)
        self.H = fock.hamiltonian(h, g, self.dets)

    def operator(self, i, tensors, bonds):
        Lmat = omps.left_basis(tensors[:i], bonds)                 # (4^i, D_i)
        Rmat = omps.right_basis(tensors[i + 2:], bonds, i + 2)     # (D_{i+2}, 4^(K-i-2))
        nl, nr = Lmat.shape[0], Rmat.shape[1]
        full = np.zeros(4 ** self.K)

        def apply(psi_dense):
            phi = np.einsum("xl,lstr,ry->xsty", Lmat, psi_dense, Rmat, optimize=True).ravel()[self.pidx]
            full[:] = 0.0
            full[self.pidx] = self.H @ phi
            return np.einsum("xl,xsty,ry->lstr", Lmat, full.reshape(nl, 4, 4, nr), Rmat, optimize=True)

        return apply


class MpoHeff:
    """H_eff = sum_{abc} L_a (x) W_i[a,b] (x) W_{i+1}[b,c] (x) R_c on dense
    zero-padded arrays (oracle.contract), environments built from the boundary
    operators at every step.  W: list of dense MPO tensors W[k][a, b, s', s] (the
    MPO values are data); the vacuum-side boundary operator and the full-chain
    boundary operator are both the 1 x 1 identity."""

    def __init__(self, W):
        self.W = [np.asarray(w, dtype=np.float64) for w in W]
        self.K = len(W)

    def environments(self, i, tensors, bonds):
        L = np.ones((1, 1, 1))
        for k in range(i):
            L = contract.env_update_left(L, self.W[k], omps.dense_site_tensor(tensors[k], bonds[k], bonds[k + 1]))
        R = np.ones((1, 1, 1))
        for k in range(self.K - 1, i + 1, -1):
            R = contract.env_update_right(R, self.W[k], omps.dense_site_tensor(tensors[k], bonds[k], bonds[k + 1]))
        return L, R

    def operator(self, i, tensors, bonds):
        L, R = self.environments(i, tensors, bonds)
        W1, W2 = self.W[i], self.W[i + 1]

        def apply(psi_dense):
            return contract.heff_apply(L, W1, W2, R, psi_dense)

        return apply


def solve_step(heff, i, tensors, bonds, psi0):
    """Lowest eigenpair of the two-site H_eff at (i, i+1) over the allowed blocks."""
    lb, rb = bonds[i], bonds[i + 2]
    keys = allowed_blocks(lb, rb)
    apply = heff.operator(i, tensors, bonds)

    def matvec(v):
        dense = omps.dense_two_site(from_vector(v, lb, rb, keys), lb, rb)
        return to_vector(omps.two_site_blocks_from_dense(apply(dense), lb, rb, keys), lb, rb, keys)

    n = sum(lb[k[0]][1] * rb[k[3]][1] for k in keys)
    v0 = to_vector(psi0, lb, rb, keys)
    energy, vec = lowest_eigenpair(matvec, n, v0)
    return energy, from_vector(vec, lb, rb, keys)


# ------------------------------------------------------------------ step 3: the split

def sector_matrices(psi, lbond, rbond):
    """psi as one dense matrix per middle-bond quantum number Q = q(il) + q(s1):
    {Q: (matrix, row labels [(il, s1, dim)], column labels [(s2, ir, dim)])}, labels
    ascending."""
    rows, cols = {}, {}
    for (il, s1, s2, ir) in psi:
        Q = _qadd(lbond[il][0], SITE_Q[s1])
        rows.setdefault(Q, set()).add((il, s1))
        cols.setdefault(Q, set()).add((s2, ir))
    out = {}
    for Q in rows:
        rl = [(il, s1, lbond[il][1]) for il, s1 in sorted(rows[Q])]
        cl = [(s2, ir, rbond[ir][1]) for s2, ir in sorted(cols[Q])]
        ro = np.cumsum([0] + [d for *_, d in rl])
        co = np.cumsum([0] + [d for *_, d in cl])
        mat = np.zeros((ro[-1], co[-1]))
        for a, (il, s1, dl) in enumerate(rl):
            for b, (s2, ir, dr) in enumerate(cl):
                blk = psi.get((il, s1, s2, ir))
                if blk is not None:
                    mat[ro[a]:ro[a + 1], co[b]:co[b + 1]] = blk
        out[Q] = (mat, rl, cl)
    return out


def select(svals, M):
    """The C8 selection: svals {Q: singular values of sector Q incl. zeros, in the
    order of the factor's columns}.  Returns {Q: number kept} and the discarded
    weight.  Order: descending value; values in a run within TIE_RTOL * s_max of the
    run's first value count as equal and are ordered by (Q, index)."""
    flat = [(float(s), Q, j) for Q in sorted(svals) for j, s in enumerate(svals[Q])]
    flat.sort(key=lambda x: -x[0])
    smax = flat[0][0] if flat else 0.0
    ordered, run = [], []
    for item in flat:
        if run and run[0][0] - item[0] > TIE_RTOL * smax:
            ordered += sorted(run, key=lambda x: (x[1], x[2]))
            run = []
        run.append(item)
    ordered += sorted(run, key=lambda x: (x[1], x[2]))
    kept = {}
    for _, Q, _ in ordered[:M]:
        kept[Q] = kept.get(Q, 0) + 1
    discarded = float(sum(s * s for s, _, _ in ordered[M:]))
    return kept, discarded


def split(psi, lbond, rbond, M, direction):
    """Split the two-site tensor at the middle bond, keeping M singular values.

    direction 0: psi = A C, A left-canonical on (il, s1), C = S V^T carried right;
    direction 1: psi = C B, B right-canonical on (s2, ir), C = U S carried left.
    Returns (new middle bond, canonical tensor, centre tensor, discarded weight,
    kept singular values sorted descending)."""
    mats = sector_matrices(psi, lbond, rbond)
    fac, svals = {}, {}
    for Q, (mat, rl, cl) in mats.items():
        U, s, Vt = np.linalg.svd(mat, full_matrices=True)
        n = U.shape[1] if direction == 0 else Vt.shape[0]   # columns of the kept square factor
        full = np.zeros(n)
        full[:len(s)] = s
        fac[Q] = (U, full, Vt, rl, cl)
        svals[Q] = full
    kept, discarded = select(svals, M)
    bond = sorted((Q, m) for Q, m in kept.items() if m > 0)
    canon, centre, ks = {}, {}, []
    for q, (Q, m) in enumerate(bond):
        U, s, Vt, rl, cl = fac[Q]
        ks += list(s[:m])
        if direction == 0:
            Vm = np.zeros((m, Vt.shape[1]))
            r = min(m, Vt.shape[0])
            Vm[:r] = Vt[:r]
            C = s[:m, None] * Vm
            o = 0
            for il, s1, d in rl:
                canon[(il, s1, q)] = U[o:o + d, :m].copy()
                o += d
            o = 0
            for s2, ir, d in cl:
                centre[(q, s2, ir)] = C[:, o:o + d].copy()
                o += d
        else:
            Um = np.zeros((U.shape[0], m))
            r = min(m, U.shape[1])
            Um[:, :r] = U[:, :r]
            C = Um * s[None, :m]
            o = 0
            for s2, ir, d in cl:
                canon[(q, s2, ir)] = Vt[:m, o:o + d].copy()
                o += d
            o = 0
            for il, s1, d in rl:
                centre[(il, s1, q)] = C[o:o + d, :].copy()
                o += d
    return bond, canon, centre, discarded, sorted(ks, reverse=True)


# ------------------------------------------------------------------ the sweep

def sweep(heff, bonds, tensors, M, n_passes):
    """Alternating two-site passes from a right-canonical MPS (bonds, tensors: copied).

    Returns the step records [{"pass", "i", "energy", "discarded", "bond", "kept_s"}],
    "bond" being the new middle bond's sector table after the step's split."""
    bonds = [list(b) for b in bonds]
    tensors = [dict(t) for t in tensors]
    K = len(tensors)
    log = []
    centre, at = None, None      # centre tensor and the site it belongs to

    def step(p, i, direction):
        nonlocal centre, at
        if centre is None:
            psi0 = merge(tensors[i], tensors[i + 1], bonds[i], bonds[i + 1], bonds[i + 2])
        elif at == i:
            psi0 = merge(centre, tensors[i + 1], bonds[i], bonds[i + 1], bonds[i + 2])
        else:
            psi0 = merge(tensors[i], centre, bonds[i], bonds[i + 1], bonds[i + 2])
        energy, psi = solve_step(heff, i, tensors, bonds, psi0)
        nb, canon, c, disc, ks = split(psi, bonds[i], bonds[i + 2], M, direction)
        bonds[i + 1] = nb
        if direction == 0:
            tensors[i], centre, at = canon, c, i + 1
        else:
            tensors[i + 1], centre, at = canon, c, i
        log.append({"pass": p, "i": i, "energy": energy, "discarded": disc, "bond": list(nb), "kept_s": ks})

    for p in range(n_passes):
        if p % 2 == 0:
            for i in range(0 if p == 0 else 1, K - 1):
                step(p, i, 0 if i < K - 2 else 1)
        else:
            for i in range(K - 3, -1, -1):
                step(p, i, 1 if i > 0 else 0)
    return log
