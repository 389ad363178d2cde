"""One-site sigma-vector (the one-site sweep's H_eff) on the GPU against the oracle.

Tolerance as for the two-site sigma-vector (FP64, 1e-11 of the largest element).
"""

import numpy as np
import pytest

from oracle import contract, mps
from synth import bond_sector_tables, make_integrals, random_left_canonical_mps, random_right_canonical_mps
from synth.blocks import random_env, random_site_ops, random_site_tensor
from test_gpu_parity import DQS, _bonds

pytestmark = pytest.mark.gpu

RTOL = 1e-11


def _check(got, ref_dense, lb, rb):
    lo, _ = mps.bond_offsets(lb)
    ro, _ = mps.bond_offsets(rb)
    scale = np.abs(ref_dense).max()
    for (il, s, ir), blk in got.items():
        ref = ref_dense[lo[il]:lo[il] + blk.shape[0], s, ro[ir]:ro[ir] + blk.shape[1]]
        assert np.abs(blk - ref).max() <= RTOL * scale, (il, s, ir)


@pytest.mark.parametrize("seed,big,variant", [(0, False, 0), (1, True, 1), (2, True, 5), (2, True, 4)])
def test_one_site_apply_and_diag_random_operands(device, seed, big, variant):
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[heff1] seed={seed} big={big} variant={variant}", flush=True)
    rng = np.random.default_rng(seed)
    lb, rb = _bonds(seed, big)
    Ldq = [DQS[i % len(DQS)] for i in range(7)]
    Rdq = [DQS[(i * 7 + 3) % len(DQS)] for i in range(7)]
    L, R = random_env(lb, Ldq, rng), random_env(rb, Rdq, rng)
    W = random_site_ops(Ldq, Rdq, rng, per_col=3)
    t = random_site_tensor(lb, rb, rng)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.Heff1Plan(lbB, rbB, Ldq, Rdq, W, kernel_variant=variant, split_kseg_min=16).upload(device)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi1(lbB, rbB, t)).to(device)
    st = torch.full_like(pt, float("nan"))
    dt = torch.full_like(pt, float("nan"))
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pt, st)
    plan.diag(Lt, Rt, dt)
    torch.cuda.synchronize()
    Ld, Wd, Rd = contract.dense_env(L, lb), contract.dense_mpo(W, len(Ldq), len(Rdq)), contract.dense_env(R, rb)
    _check(X.unpack_psi1(lbB, rbB, st.cpu().numpy()), contract.heff1_apply(Ld, Wd, Rd, mps.dense_site_tensor(t, lb, rb)),
           lb, rb)
    if not big:  # diag against the brute-force Kronecker matrix
        shape = (Ld.shape[1], 4, Rd.shape[1])
        _check(X.unpack_psi1(lbB, rbB, dt.cpu().numpy()),
               np.diag(contract.heff1_matrix_kron(Ld, Wd, Rd)).reshape(shape), lb, rb)


@pytest.mark.parametrize("i,switch", [(2, None), (4, None), (4, 4), (6, 4)])
def test_one_site_sigma_with_gpu_environments_equals_PtHP(device, i, switch):
    """MPO (NC, or NC->CN switched at cut 4) + GPU environment chain + GPU one-site
    sigma == P^T H P psi."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.engine import Engine, site_payload
    from paper_2310_03920_amd.mpo import build_mpo
    print(f"[heff1 vs PtHP] i={i} switch={switch}", flush=True)
    K, Mb = 8, 64
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, Mb)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    m = build_mpo(h, g, switch=switch)
    eng = Engine(m, device=device)
    eng.init_boundaries()
    for k in range(i):
        eng.update_left(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], left[k], device))
    for k in range(K - 1, i, -1):
        eng.update_right(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], right[k], device))
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 1])
    plan = X.Heff1Plan(lb, rb, m.dq[i], m.dq[i + 1], X.MpoSite(m.sites[i].rows, m.sites[i].cols, m.sites[i].mats))
    plan.upload(device)
    t = random_site_tensor(bonds[i], bonds[i + 1], np.random.default_rng(7))
    pt = torch.from_numpy(X.pack_psi1(lb, rb, t)).to(device)
    st = torch.empty_like(pt)
    plan.prepare(eng.left[i], eng.right[i + 1])
    plan.apply(eng.left[i], eng.right[i + 1], pt, st)
    torch.cuda.synchronize()
    emb = mps.Embedding1(h, g, K, 0, left[:i], right[i + 1:], bonds, i)
    ref = emb.apply(mps.dense_site_tensor(t, bonds[i], bonds[i + 1]))
    _check(X.unpack_psi1(lb, rb, st.cpu().numpy()), ref, bonds[i], bonds[i + 1])


@pytest.mark.parametrize("switch", [None, 3])
def test_one_site_sweep_complete_basis_gives_fci(device, switch):
    """After two-site passes at 6 orbitals, M=64 (every bond basis complete), each
    one-site step's energy is E_FCI -- with the NC MPO and with the NC->CN switch
    at cut 3 (Sec. II.B.2), whose one-site steps right of the switch see
    complementary pair operators in the left environments."""
    from oracle import fock
    from paper_2310_03920_amd.dmrg import DMRG
    print(f"[one-site sweep] K=6 complete, MPO switch {switch}", flush=True)
    K = 6
    h, g = make_integrals(K, seed=4)
    e_fci = fock.fci_energy(h, g, K, 0)
    d = DMRG(h, g, K, 0, 64, seed=3, device="cuda", tol=1e-10, max_iter=150, mpo_switch=switch)
    d.run(2)
    d.run_one_site(3)
    steps = [r for r in d.log if r.get("one_site")]
    assert len(steps) == (K - 1) + K + K
    for r in steps:
        assert abs(r["energy"] - e_fci) < 1e-9, (r, e_fci)


def test_one_site_sweep_truncated_is_variational_and_matches_embedding(device):
    """At M=12 (truncated) one-site energies never rise within the fixed bond spaces
    and stay above E_FCI; the last step's energy is the lowest eigenvalue of the
    oracle's P^T H P at that site for the final MPS."""
    from oracle import fock
    from paper_2310_03920_amd.dmrg import DMRG
    print("[one-site sweep] K=8 M=12", flush=True)
    K = 8
    h, g = make_integrals(K, seed=6)
    e_fci = fock.fci_energy(h, g, K, 0)
    d = DMRG(h, g, K, 0, 12, seed=5, device="cuda", tol=1e-10, max_iter=200)
    d.run(2)
    d.run_one_site(2)
    e = [r["energy"] for r in d.log if r.get("one_site")]
    assert all(b <= a + 1e-9 for a, b in zip(e, e[1:])), e
    assert min(e) > e_fci - 1e-10
    i = d.center_site
    assert i == 0
    emb = mps.Embedding1(h, g, K, 0, [], list(d.tensors[1:]), [list(b) for b in d.bonds], 0)
    shape = (1, 4, sum(m for _, m in d.bonds[1]))
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        v = np.zeros(n)
        v[j] = 1.0
        cols.append(emb.to_fock(v.reshape(shape)))
    P = np.array(cols).T
    keep = np.linalg.norm(P, axis=0) > 1e-12
    Pk = P[:, keep]
    Heff = Pk.T @ (emb.H @ Pk)
    assert abs(np.linalg.eigvalsh(Heff)[0] - e[-1]) < 1e-9
