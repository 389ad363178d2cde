"""Seeded full-size operands for the parity tests, laid out once in the library's
flat payload formats with the oracle's block-dict views on the same memory (no
copies), so that environments of several GB are drawn and stored only once.

Values: N(0,1) from numpy's PCG64 (seeded), drawn as whole flat payloads in the
order L, R, psi.  Structure: the middle site pair of a K-orbital chain, K
electrons, 2Sz = 0, Gaussian sector model (width 1) at bond dimension M, NC MPO of
the seeded integrals.
"""

import numpy as np

from synth import bond_sector_tables, make_integrals


def env_views(X, bond, dqs, flat):
    """The environment payload `flat` as the oracle's list of {"dq", "blocks"} whose
    blocks are views into flat."""
    op_off, blk_off = X.env_layout(bond, X.OpSet(dqs))
    sec = bond.sectors
    idx = {q: j for j, (q, _) in enumerate(sec)}
    out = []
    for a, dq in enumerate(dqs):
        blocks = {}
        for isrc, (q, n) in enumerate(sec):
            o = int(blk_off[a, isrc])
            if o < 0:
                continue
            m = sec[idx[(q[0] + dq[0], q[1] + dq[1])]][1]
            blocks[isrc] = flat[o:o + m * n].reshape(m, n)
        out.append({"dq": tuple(dq), "blocks": blocks})
    return out


def psi_views(X, lbond, rbond, flat):
    keys, off = X.psi_layout(lbond, rbond)
    return {k: flat[int(off[j]):int(off[j + 1])].reshape(lbond.sectors[k[0]][1], rbond.sectors[k[3]][1])
            for j, k in enumerate(keys)}


def middle_problem(X, K, M, seed=2024):
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    i = K // 2 - 1
    mpo = build_nc_mpo(*make_integrals(K, seed=0))
    bonds = bond_sector_tables(K, K, 0, M, model="gaussian", width=1.0)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    Ldq = [tuple(int(v) for v in x) for x in mpo.dq[i]]
    Mdq = [tuple(int(v) for v in x) for x in mpo.dq[i + 1]]
    Rdq = [tuple(int(v) for v in x) for x in mpo.dq[i + 2]]
    nL = int(X.env_layout(lb, X.OpSet(Ldq))[0][-1])
    nR = int(X.env_layout(rb, X.OpSet(Rdq))[0][-1])
    nP = int(X.psi_layout(lb, rb)[1][-1])
    rng = np.random.default_rng(seed)
    Lf, Rf, Pf = rng.standard_normal(nL), rng.standard_normal(nR), rng.standard_normal(nP)
    W1 = X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats)
    W2 = X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats)
    return dict(K=K, M=M, i=i, mpo=mpo, bonds=bonds, lb=lb, rb=rb, Ldq=Ldq, Mdq=Mdq, Rdq=Rdq,
                Lf=Lf, Rf=Rf, Pf=Pf, L=env_views(X, lb, Ldq, Lf), R=env_views(X, rb, Rdq, Rf),
                psi=psi_views(X, lb, rb, Pf), W1=W1, W2=W2,
                W1e=site_entries(mpo, i), W2e=site_entries(mpo, i + 1))


def sample_rows(lbond, count=6, seed=5):
    """Rows (il', s1', x) of sigma: the first and last rows of the largest left sector
    (the last one in a ragged 64-row tile), a row of the smallest, then random."""
    sec = lbond.sectors if hasattr(lbond, "sectors") else lbond
    big = max(range(len(sec)), key=lambda j: sec[j][1])
    one = min(range(len(sec)), key=lambda j: sec[j][1])
    rows = [(big, 1, 0), (big, 2, sec[big][1] - 1), (one, 0, 0)]
    pick = np.random.default_rng(seed)
    while len(rows) < count:
        il = int(pick.integers(len(sec)))
        rows.append((il, int(pick.integers(4)), int(pick.integers(sec[il][1]))))
    return rows


def compare_rows(X, lb, rb, sigma_host, ref):
    """max |gpu - oracle| over the sampled rows, and the scale max |oracle|."""
    got = psi_views(X, lb, rb, sigma_host)
    worst, scale = 0.0, 0.0
    for (il, s1, x), cols in ref.items():
        for (s2, ir), vec in cols.items():
            worst = max(worst, float(np.max(np.abs(got[(il, s1, s2, ir)][x] - vec))))
            scale = max(scale, float(np.max(np.abs(vec))))
    return worst, scale
