"""Block-sparse sigma-vector on the host, by blocks (TEST INFRASTRUCTURE ONLY).

The renormalised-operator form of the two-site H_eff (Sec. II.C.1: the MPO
multiplication reproduces the DMRG equations; Sec. II.A.1: symmetry blocks make
every product a dense product of blocks):

  sigma = sum_b  Lhat_b  psi  Rhat_b^T,
  Lhat_b[s1' <- s1] = sum_a W1[a, b][s1', s1] L_a,
  Rhat_b[s2' <- s2] = sum_c W2[b, c][s2', s2] R_c,

evaluated on dicts of dense blocks: for every output column block (s2', r') and
every middle-bond index b, first the intermediate
  T_b[l, s1 | s2', r'] = sum_{s2, r} psi[l, s1, s2, r] Rhat_b[s2' <- s2][r' <- r]^T,
then
  sigma[l', s1' | s2', r'] += sum_{s1, l} Lhat_b[s1' <- s1][l' <- l] T_b[l, s1 | s2', r'].
Each block product m x k times k x n is one numpy matmul and is counted as 2 m n k
floating-point operations (the method's own work: blocks the symmetry forbids,
zero site-matrix entries and intermediate blocks that the second product does not read are
never touched; forming Lhat / Rhat is counted apart).
`bsel` restricts the sum to a subset of b (the terms of different b are
independent, so sigma is the sum of the restricted results over a partition of b).

Formats are those of the synth package: environments as lists of
{"dq": (dN, d2Sz), "blocks": {source sector: block}}, MPO entries as (row, col,
4x4 matrix), psi as {(il, s1, s2, ir): block}.
"""

def mixed_operators(env, entries, by_row, bsel=None):
    """{b: {(s_out, s_in): {src: (dst, block)}}}: sum over the coupled environment
    operators of the site-matrix element times the operator's blocks.  by_row: the
    environment index is the entry's row (left: W1[a, b]) or its column (right:
    W2[b, c]); b is the other index.  bsel: only these b (None = all)."""
    out = {}
    keep = None if bsel is None else set(bsel)
    for row, col, op in entries:
        a, b = (row, col) if by_row else (col, row)
        if keep is not None and b not in keep:
            continue
        dq = env[a]["dq"]
        for so in range(4):
            for si in range(4):
                w = op[so, si]
                if w == 0.0:
                    continue
                tgt = out.setdefault(b, {}).setdefault((so, si), {})
                for src, blk in env[a]["blocks"].items():
                    if src in tgt:
                        if tuple(tgt[src][0]) != tuple(dq):
                            raise ValueError("MPO entries of one (b, s', s) couple operators of different shifts")
                        tgt[src] = (tgt[src][0], tgt[src][1] + w * blk)
                    else:
                        tgt[src] = (dq, w * blk)
    return out


def prepare(L, W1e, W2e, R, bsel=None):
    """The mixed operators (Lhat, Rhat) of the middle-bond indices in bsel."""
    return mixed_operators(L, W1e, True, bsel), mixed_operators(R, W2e, False, bsel)


def heff_apply(lbond, rbond, L, W1e, W2e, R, psi, bsel=None, cols=None, flops=None, mixed=None):
    """sigma blocks {(il', s1', s2', ir'): block} (only blocks that receive a term).

    bsel: iterable of middle-bond indices to include (None = all); cols: output
    column blocks (s2', ir') to compute (None = all); flops: a one-element list that
    receives the count of 2 m n k over the block products; mixed: the result of
    prepare() for the same operands and bsel (computed here when None)."""
    lidx = {q: j for j, (q, _) in enumerate(lbond)}
    ridx = {q: j for j, (q, _) in enumerate(rbond)}
    Lhat, Rhat = mixed if mixed is not None else prepare(L, W1e, W2e, R, bsel)
    bs = sorted(set(Lhat) & set(Rhat))
    if bsel is not None:
        keep = set(bsel)
        bs = [b for b in bs if b in keep]
    psi_by_s2 = {}
    for (il, s1, s2, ir), blk in psi.items():
        psi_by_s2.setdefault(s2, []).append((il, s1, ir, blk))
    if cols is None:
        cols = sorted({(s2, ir) for (_, _, s2, ir) in psi})
    # row blocks (il, s1) of T_b that the second product reads: some left transition of b starts
    # from s1 and its mixed operator has a block with source il
    reads = {b: {(il, si) for (so, si), ops in Lhat[b].items() for il in ops} for b in bs}
    count = 0.0
    sigma = {}
    for (s2p, irp) in cols:
        for b in bs:
            # first product: T_b[(il, s1)] for this output column block
            T = {}
            for (so, si), ops in Rhat[b].items():
                if so != s2p:
                    continue
                for il, s1, ir, blk in psi_by_s2.get(si, []):
                    if (il, s1) not in reads[b]:
                        continue
                    hit = ops.get(ir)
                    if hit is None:
                        continue
                    dq, rblk = hit
                    qr = rbond[ir][0]
                    if ridx.get((qr[0] + dq[0], qr[1] + dq[1])) != irp:
                        continue
                    prod = blk @ rblk.T
                    count += 2.0 * blk.shape[0] * blk.shape[1] * rblk.shape[0]
                    T[(il, s1)] = T[(il, s1)] + prod if (il, s1) in T else prod
            if not T:
                continue
            # second product: sigma[(il', s1', s2', ir')] += Lhat_b[s1' <- s1][il' <- il] T_b[(il, s1)]
            for (so, si), ops in Lhat[b].items():
                for (il, s1), t in T.items():
                    if s1 != si:
                        continue
                    hit = ops.get(il)
                    if hit is None:
                        continue
                    dq, lblk = hit
                    ql = lbond[il][0]
                    ilp = lidx.get((ql[0] + dq[0], ql[1] + dq[1]))
                    if ilp is None:
                        continue
                    prod = lblk @ t
                    count += 2.0 * lblk.shape[0] * lblk.shape[1] * t.shape[1]
                    key = (ilp, so, s2p, irp)
                    sigma[key] = sigma[key] + prod if key in sigma else prod
    if flops is not None:
        flops[0] += count
    return sigma
