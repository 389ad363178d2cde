"""MPS -> Fock-space embedding and the definition H_eff := P^T H P (Sec. II.A.2).

For the two-site step at sites (i, i+1) the renormalised wavefunction
psi[l, s1, s2, r] lives in the product of the left block basis (bond i), two
site bases and the right block basis (bond i+2).  The left basis states are
columns of the contracted left-canonical tensors A_0..A_{i-1}, the right basis
states rows of the contracted right-canonical tensors B_{i+2}..B_{K-1}; together
they define an isometry P from the two-site space into Fock space, and the
effective Hamiltonian of the sweep is H_eff = P^T H P.  This module computes that
definition directly: no MPO and no environments are involved.

The site-product basis |s_0 ... s_{K-1}> (s_0 most significant) equals the
determinant basis of oracle.fock with no extra sign (see fock.product_index).
"""

import numpy as np

from . import fock


def bond_offsets(bond):
    offs, o = [], 0
    for _, m in bond:
        offs.append(o)
        o += m
    return offs, o


def dense_site_tensor(t, lbond, rbond):
    lo, dl = bond_offsets(lbond)
    ro, dr = bond_offsets(rbond)
    out = np.zeros((dl, 4, dr))
    for (il, s, ir), blk in t.items():
        out[lo[il]:lo[il] + blk.shape[0], s, ro[ir]:ro[ir] + blk.shape[1]] = blk
    return out


def dense_two_site(psi, lbond, rbond):
    lo, dl = bond_offsets(lbond)
    ro, dr = bond_offsets(rbond)
    out = np.zeros((dl, 4, 4, dr))
    for (il, s1, s2, ir), blk in psi.items():
        out[lo[il]:lo[il] + blk.shape[0], s1, s2, ro[ir]:ro[ir] + blk.shape[1]] = blk
    return out


def two_site_blocks_from_dense(arr, lbond, rbond, keys):
    lo, _ = bond_offsets(lbond)
    ro, _ = bond_offsets(rbond)
    out = {}
    for (il, s1, s2, ir) in keys:
        ml, mr = lbond[il][1], rbond[ir][1]
        out[(il, s1, s2, ir)] = arr[lo[il]:lo[il] + ml, s1, s2, ro[ir]:ro[ir] + mr].copy()
    return out


def left_basis(tensors, bonds):
    """Rows: site-product index of (s_0..s_{i-1}); columns: bond-i basis states."""
    m = np.ones((1, 1))
    for k, t in enumerate(tensors):
        a = dense_site_tensor(t, bonds[k], bonds[k + 1])  # (Dl, 4, Dr)
        m = np.einsum("xl,lsr->xsr", m, a).reshape(m.shape[0] * 4, a.shape[2])
    return m


def right_basis(tensors, bonds, first):
    """Rows: bond-`first` basis states; columns: site-product index of the sites."""
    m = np.ones((1, 1))
    for k in range(len(tensors) - 1, -1, -1):
        b = dense_site_tensor(tensors[k], bonds[first + k], bonds[first + k + 1])  # (Dl, 4, Dr)
        m = np.einsum("lsr,ry->lsy", b, m).reshape(b.shape[0], 4 * m.shape[1])
    return m


class Embedding:
    """P for the two-site step at (i, i+1), restricted to the target sector."""

    def __init__(self, h, g, N, twosz, left_tensors, right_tensors, bonds, i):
        K = h.shape[0]
        self.K, self.i, self.bonds = K, i, bonds
        self.Lmat = left_basis(left_tensors, bonds)                  # (4^i, D_i)
        self.Rmat = right_basis(right_tensors, bonds, i + 2)        # (D_{i+2}, 4^{K-i-2})
        self.dets = fock.sector_dets(K, N, twosz)
        self.pidx = fock.product_index(self.dets, K)
        self.H = fock.hamiltonian(h, g, self.dets)

    def to_fock(self, psi_dense):
        phi = np.einsum("xl,lstr,ry->xsty", self.Lmat, psi_dense, self.Rmat)
        return phi.ravel()[self.pidx]

    def from_fock(self, vec):
        full = np.zeros(4 ** self.K)
        full[self.pidx] = vec
        nl, nr = self.Lmat.shape[0], self.Rmat.shape[1]
        phi = full.reshape(nl, 4, 4, nr)
        return np.einsum("xl,xsty,ry->lstr", self.Lmat, phi, self.Rmat)

    def apply(self, psi_dense):
        """sigma = P^T H P psi on dense (D_i, 4, 4, D_{i+2}) arrays."""
        return self.from_fock(self.H @ self.to_fock(psi_dense))

    def embedding_matrix(self, keys):
        """P restricted to the sector: rows = sector determinants, columns = the
        elements of the listed two-site blocks (block order = keys, row-major)."""
        lb, rb = self.bonds[self.i], self.bonds[self.i + 2]
        lo, _ = bond_offsets(lb)
        ro, _ = bond_offsets(rb)
        nr = self.Rmat.shape[1]
        x = self.pidx // (16 * nr)
        d1 = (self.pidx // (4 * nr)) % 4
        d2 = (self.pidx // nr) % 4
        y = self.pidx % nr
        cols = []
        for (il, s1, s2, ir) in keys:
            L = self.Lmat[:, lo[il]:lo[il] + lb[il][1]]          # (4^i, ml)
            R = self.Rmat[ro[ir]:ro[ir] + rb[ir][1], :]          # (mr, 4^..)
            sel = ((d1 == s1) & (d2 == s2)).astype(float)
            c = L[x][:, :, None] * R[:, y].T[:, None, :] * sel[:, None, None]
            cols.append(c.reshape(len(self.pidx), -1))
        return np.concatenate(cols, axis=1)

    def heff_matrix(self, keys):
        """Dense P^T H P over the listed two-site blocks."""
        P = self.embedding_matrix(keys)
        return P.T @ (self.H @ P)


class Embedding1:
    """P for the one-site step at site i (left basis x site x right basis), restricted
    to the target sector: H_eff := P^T H P by definition, without an MPO."""

    def __init__(self, h, g, N, twosz, left_tensors, right_tensors, bonds, i):
        K = h.shape[0]
        self.K, self.i, self.bonds = K, i, bonds
        self.Lmat = left_basis(left_tensors, bonds)              # (4^i, D_i)
        self.Rmat = right_basis(right_tensors, bonds, i + 1)    # (D_{i+1}, 4^{K-i-1})
        self.dets = fock.sector_dets(K, N, twosz)
        self.pidx = fock.product_index(self.dets, K)
        self.H = fock.hamiltonian(h, g, self.dets)

    def to_fock(self, psi1_dense):
        phi = np.einsum("xl,lsr,ry->xsy", self.Lmat, psi1_dense, self.Rmat)
        return phi.ravel()[self.pidx]

    def from_fock(self, vec):
        full = np.zeros(4 ** self.K)
        full[self.pidx] = vec
        phi = full.reshape(self.Lmat.shape[0], 4, self.Rmat.shape[1])
        return np.einsum("xl,xsy,ry->lsr", self.Lmat, phi, self.Rmat)

    def apply(self, psi1_dense):
        """sigma = P^T H P psi on dense (D_i, 4, D_{i+1}) arrays."""
        return self.from_fock(self.H @ self.to_fock(psi1_dense))
