"""Renormalised-operator contractions of the two-site sweep, by definition.

With the MPO written as operator-valued matrices W^(k) whose site operators
already carry the Jordan-Wigner parity strings, every product below is a plain
tensor (Kronecker) product, so the paper's "MPO multiplication reproducing the
DMRG equations" (Sec. II.C.1) becomes:

  sigma[l', s1', s2', r'] = sum_{a,b,c} sum_{l,s1,s2,r}
        L_a[l', l] W1_ab[s1', s1] W2_bc[s2', s2] R_c[r', r] psi[l, s1, s2, r]

  L'_b[m, n] = sum_{a, s, t, x, y} A[x, s, m] L_a[x, y] W_ab[s, t] A[y, t, n]
  R'_a[m, n] = sum_{b, s, t, x, y} B[m, s, x] W_ab[s, t] R_b[x, y] B[n, t, y]

  diag(H_eff)[l, s1, s2, r] = sum_{a,b,c} L_a[l,l] W1_ab[s1,s1] W2_bc[s2,s2] R_c[r,r]

Each is evaluated on dense zero-padded arrays as a chain of pairwise einsum
contractions, one summed index group at a time (psi with L, then W1, W2, R);
this only uses associativity of the single sum above, with no blocking.  `sigma_rows` evaluates selected
output rows of the first formula at full size, summing over b in order.
"""

import numpy as np

from .mps import bond_offsets


def dense_env(ops, bond):
    offs, D = bond_offsets(bond)
    idx = {q: i for i, (q, _) in enumerate(bond)}
    out = np.zeros((len(ops), D, D))
    for a, op in enumerate(ops):
        for isrc, blk in op["blocks"].items():
            q = bond[isrc][0]
            idst = idx[(q[0] + op["dq"][0], q[1] + op["dq"][1])]
            out[a, offs[idst]:offs[idst] + blk.shape[0], offs[isrc]:offs[isrc] + blk.shape[1]] = blk
    return out


def env_blocks_from_dense(arr, bond, dqs):
    offs, _ = bond_offsets(bond)
    idx = {q: i for i, (q, _) in enumerate(bond)}
    ops = []
    for a, dq in enumerate(dqs):
        blocks = {}
        for isrc, (q, m) in enumerate(bond):
            qd = (q[0] + dq[0], q[1] + dq[1])
            if qd in idx:
                idst = idx[qd]
                blocks[isrc] = arr[a, offs[idst]:offs[idst] + bond[idst][1], offs[isrc]:offs[isrc] + m].copy()
        ops.append({"dq": tuple(dq), "blocks": blocks})
    return ops


def dense_mpo(entries, nrow, ncol):
    w = np.zeros((nrow, ncol, 4, 4))
    for a, b, op in entries:
        w[a, b] += op
    return w


def heff_apply(Ld, W1, W2, Rd, psi):
    """sigma for dense L[a,l',l], W1[a,b,s',s], W2[b,c,t',t], R[c,r',r], psi[l,s,t,r]."""
    x = np.einsum("axy,ytvw->axtvw", Ld, psi, optimize=True)
    y = np.einsum("abst,axtvw->bxsvw", W1, x, optimize=True)
    z = np.einsum("bcuv,bxsvw->cxsuw", W2, y, optimize=True)
    return np.einsum("czw,cxsuw->xsuz", Rd, z, optimize=True)


def heff1_apply(Ld, W, Rd, psi1):
    """One-site sigma (the one-site sweep, Sec. II.A.2) for dense L[a,l',l], W[a,b,s',s],
    R[b,r',r], psi1[l,s,r]:  sigma[x,s,z] = sum L[a,x,y] W[a,b,s,t] R[b,z,w] psi1[y,t,w]."""
    x = np.einsum("axy,ytw->axtw", Ld, psi1, optimize=True)
    y = np.einsum("abst,axtw->bxsw", W, x, optimize=True)
    return np.einsum("bzw,bxsw->xsz", Rd, y, optimize=True)


def heff1_matrix_kron(Ld, W, Rd):
    """Brute force: H_eff = sum_ab kron(L_a, W_ab, R_b) (tiny sizes only)."""
    n = Ld.shape[1] * 4 * Rd.shape[1]
    H = np.zeros((n, n))
    for a in range(Ld.shape[0]):
        for b in range(W.shape[1]):
            if np.any(W[a, b]):
                H += np.kron(np.kron(Ld[a], W[a, b]), Rd[b])
    return H


def heff_vjp(Ld, W1, W2, Rd, psi, g):
    """Vector-Jacobian products of sigma = heff_apply(L, W1, W2, R, psi) with the
    cotangent g[x,s,u,z]: the derivatives of <g, sigma> with respect to each
    operand, from the same single sum differentiated term by term:

      d/dpsi[y,t,v,w] = sum g[x,s,u,z] L[a,x,y] W1[a,b,s,t] W2[b,c,u,v] R[c,z,w]
      d/dL[a,x,y]     = sum g[x,s,u,z] W1[a,b,s,t] W2[b,c,u,v] R[c,z,w] psi[y,t,v,w]
      d/dW1[a,b,s,t]  = sum g[x,s,u,z] L[a,x,y] W2[b,c,u,v] R[c,z,w] psi[y,t,v,w]
      d/dW2[b,c,u,v]  = sum g[x,s,u,z] L[a,x,y] W1[a,b,s,t] R[c,z,w] psi[y,t,v,w]
      d/dR[c,z,w]     = sum g[x,s,u,z] L[a,x,y] W1[a,b,s,t] W2[b,c,u,v] psi[y,t,v,w]

    Returns (g_L, g_W1, g_W2, g_R, g_psi) as dense arrays."""
    # cotangent carried through L, W1, W2 (the left part of each product)
    p = np.einsum("axy,xsuz->aysuz", Ld, g, optimize=True)
    q = np.einsum("abst,aysuz->bytuz", W1, p, optimize=True)
    r = np.einsum("bcuv,bytuz->cytvz", W2, q, optimize=True)
    g_psi = np.einsum("czw,cytvz->ytvw", Rd, r, optimize=True)
    g_R = np.einsum("cytvz,ytvw->czw", r, psi, optimize=True)
    # psi carried through R, W2 (the right part of each product)
    m1 = np.einsum("czw,ytvw->cytvz", Rd, psi, optimize=True)
    m2 = np.einsum("bcuv,cytvz->bytuz", W2, m1, optimize=True)
    g_W2 = np.einsum("bytuz,cytvz->bcuv", q, m1, optimize=True)
    g_W1 = np.einsum("aysuz,bytuz->abst", p, m2, optimize=True)
    m3 = np.einsum("abst,bytuz->aysuz", W1, m2, optimize=True)
    g_L = np.einsum("xsuz,aysuz->axy", g, m3, optimize=True)
    return g_L, g_W1, g_W2, g_R, g_psi


def heff_diag(Ld, W1, W2, Rd):
    dl = np.einsum("axx->ax", Ld)
    dw1 = np.einsum("abss->abs", W1)
    dw2 = np.einsum("bcuu->bcu", W2)
    dr = np.einsum("czz->cz", Rd)
    left = np.einsum("ax,abs->bxs", dl, dw1, optimize=True)
    right = np.einsum("bcu,cz->buz", dw2, dr, optimize=True)
    return np.einsum("bxs,buz->xsuz", left, right, optimize=True)


def heff_matrix_kron(Ld, W1, W2, Rd):
    """Brute force: H_eff = sum_abc kron(L_a, W1_ab, W2_bc, R_c) (tiny sizes only)."""
    n = Ld.shape[1] * 16 * Rd.shape[1]
    H = np.zeros((n, n))
    for a in range(Ld.shape[0]):
        for b in range(W1.shape[1]):
            if not np.any(W1[a, b]):
                continue
            for c in range(Rd.shape[0]):
                if not np.any(W2[b, c]):
                    continue
                H += np.kron(np.kron(np.kron(Ld[a], W1[a, b]), W2[b, c]), Rd[c])
    return H


def env_update_left(Ld, W, A):
    """L'_b = sum A^T (L_a (x) W_ab) A with A[l, s, m] (dense)."""
    t = np.einsum("axy,ytn->axtn", Ld, A, optimize=True)
    u = np.einsum("abst,axtn->bxsn", W, t, optimize=True)
    return np.einsum("xsm,bxsn->bmn", A, u, optimize=True)


def env_update_right(Rd, W, B):
    """R'_a = sum B (W_ab (x) R_b) B^T with B[m, s, x] (dense)."""
    t = np.einsum("bxy,nty->bxnt", Rd, B, optimize=True)
    u = np.einsum("abst,bxnt->axsn", W, t, optimize=True)
    return np.einsum("msx,axsn->amn", B, u, optimize=True)


def sigma_rows(lbond, rbond, L, W1e, W2e, R, psi, rows):
    """Selected rows of sigma at any size, straight from the block formats.

    rows: list of (il', s1', x) -- left sector, first site state, row within block.
    Returns {(il', s1', x): {(s2', ir'): row vector of length dim(ir')}}.
    Sums run over b in increasing order; within b over (a, s1) then (c, s2).
    """
    lidx = {q: i for i, (q, _) in enumerate(lbond)}
    ridx = {q: i for i, (q, _) in enumerate(rbond)}
    by_b1 = {}
    for a, b, op in W1e:
        by_b1.setdefault(b, []).append((a, op))
    by_b2 = {}
    for b, c, op in W2e:
        by_b2.setdefault(b, []).append((c, op))
    psi_by_l = {}
    for (il, s1, s2, ir), blk in psi.items():
        psi_by_l.setdefault((il, s1), []).append((s2, ir, blk))
    out = {}
    for (ilp, s1p, x) in rows:
        qlp = lbond[ilp][0]
        acc = {}
        for b in sorted(set(by_b1) & set(by_b2)):
            # u_b[(il, s1)] = sum_a W1_ab[s1', s1] L_a[l' <- l][x, :]
            u = {}
            for a, op in by_b1[b]:
                dq = L[a]["dq"]
                ql = (qlp[0] - dq[0], qlp[1] - dq[1])
                if ql not in lidx:
                    continue
                il = lidx[ql]
                if il not in L[a]["blocks"]:
                    continue
                lrow = L[a]["blocks"][il][x]
                for s1 in range(4):
                    if op[s1p, s1] != 0.0:
                        key = (il, s1)
                        u[key] = u.get(key, 0.0) + op[s1p, s1] * lrow
            if not u:
                continue
            # v_b[(s2, ir)] = sum_{il,s1} u . psi[il, s1, s2, ir]
            v = {}
            for (il, s1), vec in u.items():
                for s2, ir, blk in psi_by_l.get((il, s1), []):
                    v[(s2, ir)] = v.get((s2, ir), 0.0) + vec @ blk
            # acc[(s2', ir')] += sum_{c,s2} W2_bc[s2', s2] v[(s2, ir)] R_c[r' <- r]^T
            for c, op in by_b2[b]:
                dq = R[c]["dq"]
                for (s2, ir), vec in v.items():
                    if ir not in R[c]["blocks"]:
                        continue
                    qr = rbond[ir][0]
                    irp = ridx.get((qr[0] + dq[0], qr[1] + dq[1]))
                    if irp is None:
                        continue
                    contrib = R[c]["blocks"][ir] @ vec
                    for s2p in range(4):
                        if op[s2p, s2] != 0.0:
                            acc[(s2p, irp)] = acc.get((s2p, irp), 0.0) + op[s2p, s2] * contrib
        out[(ilp, s1p, x)] = acc
    return out


def env_rows_left(bond_in, bond_out, L, We, A, rows):
    """Selected rows of the left update L'_b[m, n] = sum_{a,s,t,x,y} A[x,s,m] L_a[x,y]
    W_ab[s,t] A[y,t,n], at any size, straight from the block formats.

    bond_in: bond k (L's bond); bond_out: bond k+1; L: environment on bond_in; We: MPO
    entries (a, b, op) of site k; A: site tensor {(il, s, iq): block (dim il x dim iq)}.
    rows: list of (b, iq, m) -- output operator, its row sector on bond_out, row.
    Returns {(b, iq, m): {iq_n: row vector over sector iq_n}}; sums run over the MPO
    entries in order, then s, t, then the blocks of A in key order."""
    by_b = {}
    for a, b, op in We:
        by_b.setdefault(b, []).append((a, op))
    idx_in = {q: j for j, (q, _) in enumerate(bond_in)}
    out = {}
    for (b, iq, m) in rows:
        acc = {}
        for a, op in by_b.get(b, []):
            dq = L[a]["dq"]
            for (ilx, s, iqm), blk in A.items():
                if iqm != iq:
                    continue
                u = blk[:, m]                                   # over x in sector ilx
                q = bond_in[ilx][0]
                ily = idx_in.get((q[0] - dq[0], q[1] - dq[1]))  # L_a maps ily -> ilx
                if ily is None or ily not in L[a]["blocks"]:
                    continue
                v = u @ L[a]["blocks"][ily]                     # over y in sector ily
                for t in range(4):
                    w = op[s, t]
                    if w == 0.0:
                        continue
                    for (ily2, t2, iqn), blk2 in A.items():
                        if ily2 == ily and t2 == t:
                            acc[iqn] = acc.get(iqn, 0.0) + w * (v @ blk2)
        out[(b, iq, m)] = acc
    return out


def env_rows_right(bond_in, bond_out, R, We, B, rows):
    """Selected rows of the right update R'_a[m, n] = sum_{b,s,t,x,y} B[m,s,x] W_ab[s,t]
    R_b[x,y] B[n,t,y], at any size, straight from the block formats.

    bond_in: bond k+1 (R's bond); bond_out: bond k; R: environment on bond_in; We: MPO
    entries (a, b, op) of site k; B: site tensor {(iq, s, ix): block (dim iq x dim ix)}.
    rows: list of (a, iq, m) -- output operator, its row sector on bond_out, row.
    Returns {(a, iq, m): {iq_n: row vector over sector iq_n}}."""
    by_a = {}
    for a, b, op in We:
        by_a.setdefault(a, []).append((b, op))
    idx_in = {q: j for j, (q, _) in enumerate(bond_in)}
    out = {}
    for (a, iq, m) in rows:
        acc = {}
        for b, op in by_a.get(a, []):
            dq = R[b]["dq"]
            for (iqm, s, ix), blk in B.items():
                if iqm != iq:
                    continue
                u = blk[m, :]                                   # over x in sector ix
                q = bond_in[ix][0]
                iy = idx_in.get((q[0] - dq[0], q[1] - dq[1]))   # R_b maps iy -> ix
                if iy is None or iy not in R[b]["blocks"]:
                    continue
                v = u @ R[b]["blocks"][iy]                      # over y in sector iy
                for t in range(4):
                    w = op[s, t]
                    if w == 0.0:
                        continue
                    for (iqn, t2, iy2), blk2 in B.items():
                        if iy2 == iy and t2 == t:
                            acc[iqn] = acc.get(iqn, 0.0) + w * (blk2 @ v)
        out[(a, iq, m)] = acc
    return out
