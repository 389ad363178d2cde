"""FP32 and BF16 precision modes of the block contractions (Davidson stays FP64).

Parity of the FP32 sigma-vector is unpinned except relative to FP64: each input
is rounded once to FP32 (relative 2^-24) and the products are accumulated in
FP32 (MFMA f32 accumulation) over at most ~2e3 terms here, so an element can
differ from the FP64 definition by at most ~2e3 * 2^-24 * sum|terms|; the test
bound is 2e-4 of the largest reference element.  Energies are pinned: the mixed
Davidson refines the FP32 Ritz vector with FP64 sigma-vectors, so its energy
must equal the FP64 eigenvalue to 1e-10 Ha.

BF16 products: every operand is rounded once to BF16 when staged (relative
2^-9), T again before the second round, so a product carries at most ~4 * 2^-9
relative error; these errors are independent between terms and add like the
terms themselves, so an element lands within a few 2^-7 of the largest
reference element: the bound is 2e-2.
"""

import numpy as np
import pytest

from oracle import fock, mps
from synth import bond_sector_tables, make_integrals, random_left_canonical_mps, random_right_canonical_mps
from synth.blocks import random_psi, two_site_blocks

from test_gpu_parity import _close, _dense_sigma, _problem

pytestmark = pytest.mark.gpu

RTOL32 = 2e-4
RTOL_BF16 = 2e-2


def _f32_sigma(device, prob, bf16=False):
    import torch
    from paper_2310_03920_amd import _lib as X
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, split_kseg_min=32).upload(device)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    plan.prepare(Lt, Rt)
    plan.lower_f32(Lt, Rt)
    p32 = torch.empty(pt.numel(), dtype=torch.float32, device=device)
    s32 = torch.full_like(p32, float("nan"))
    X.convert_f64_f32(pt, p32)
    low = plan.apply_bf16 if bf16 else plan.apply_f32
    low(p32, s32)
    s64 = torch.empty_like(pt)
    X.convert_f32_f64(s32, s64)
    s32b = torch.empty_like(p32)
    low(p32, s32b)
    torch.cuda.synchronize()
    assert torch.equal(s32, s32b)
    return X.unpack_psi(lbB, rbB, s64.cpu().numpy())


@pytest.mark.parametrize("seed", [1, 2])
def test_heff_apply_f32_random_operands(device, seed):
    print(f"[heff_apply_f32] seed={seed}", flush=True)
    prob = _problem(seed, True)
    _close(_f32_sigma(device, prob), _dense_sigma(*prob), rtol=RTOL32)


@pytest.mark.parametrize("seed", [1, 2])
def test_heff_apply_bf16_random_operands(device, seed):
    print(f"[heff_apply_bf16] seed={seed}", flush=True)
    prob = _problem(seed, True)
    _close(_f32_sigma(device, prob, bf16=True), _dense_sigma(*prob), rtol=RTOL_BF16)


def test_mixed_davidson_reaches_fp64_energy(device):
    """Middle step of the 8-orbital problem with GPU environments: the mixed
    FP32/FP64 Davidson energy equals the FP64 Davidson energy and the lowest
    eigenvalue of the oracle's P^T H P."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.dmrg import Davidson
    from paper_2310_03920_amd.engine import Engine, site_payload
    from paper_2310_03920_amd.mpo import build_nc_mpo
    print("[mixed davidson]", flush=True)
    K, i = 8, 3
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, 64)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    eng = Engine(build_nc_mpo(h, g), device=device)
    eng.init_boundaries()
    for k in range(i):
        eng.update_left(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], left[k], device))
    for k in range(K - 1, i + 1, -1):
        eng.update_right(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], right[k], device))
    plan = eng.heff_plan(i, bonds[i], bonds[i + 2])
    L, R = eng.left[i], eng.right[i + 2]
    n = int(plan.info.psi_nnz)
    plan.prepare(L, R)
    plan.lower_f32(L, R)
    diag = torch.empty(n, dtype=torch.float64, device=device)
    plan.diag(L, R, diag)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    psi0 = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], np.random.default_rng(5)))).to(device)
    v32 = torch.empty(n, dtype=torch.float32, device=device)
    s32 = torch.empty_like(v32)

    def mv(v, out):
        plan.apply(L, R, v, out)

    def mv32(v, out):
        X.convert_f64_f32(v, v32)
        plan.apply_f32(v32, s32)
        X.convert_f32_f64(s32, out)

    def mvb(v, out):
        X.convert_f64_f32(v, v32)
        plan.apply_bf16(v32, s32)
        X.convert_f32_f64(s32, out)

    dav = Davidson(n, 24, device)
    e64, r64, _ = dav.solve(mv, psi0, diag, tol=1e-9, max_iter=200)
    e32, _, _ = Davidson(n, 24, device).solve(mv32, psi0, diag, tol=1e-5, max_iter=200)
    em, rm, n32, n64 = Davidson(n, 24, device).solve_mixed(mv32, mv, psi0, diag, tol=1e-9, max_iter=200)
    eb, rb_, nb16, nb64 = Davidson(n, 24, device).solve_mixed(mvb, mv, psi0, diag, tol=1e-9, max_iter=200,
                                                              low_tol=3e-3)
    print(f"bf16 mixed: E {eb:.12f} ({nb16} bf16 + {nb64} f64 matvecs)", flush=True)
    assert rb_ < 1e-9 and abs(eb - e64) < 1e-10
    # a warm start already below what BF16 products resolve: the BF16 phase gives up
    # within a few iterations instead of running to max_iter
    ew, rw, nw16, nw64 = Davidson(n, 24, device).solve_mixed(mvb, mv, dav.x.clone(), diag, tol=1e-9, max_iter=200,
                                                             low_tol=1e-12)
    print(f"bf16 mixed from the converged vector: {nw16} bf16 + {nw64} f64 matvecs", flush=True)
    assert nw16 <= 16 and rw < 1e-9 and abs(ew - e64) < 1e-10
    e_fci = fock.fci_energy(h, g, K, 0)
    print(f"E64 {e64:.12f} E32-only {e32:.12f} Emixed {em:.12f} FCI {e_fci:.12f} (f32 {n32}, f64 {n64} matvecs)",
          flush=True)
    assert r64 < 1e-9 and rm < 1e-9
    assert abs(e64 - e_fci) < 1e-10
    assert abs(em - e64) < 1e-10
    assert abs(e32 - e64) < 1e-4      # FP32-only energy: within the FP32 rounding floor


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_mixed_precision_sweep_matches_fci(device, precision):
    from paper_2310_03920_amd.dmrg import DMRG
    print(f"[sweep {precision}]", flush=True)
    K = 8
    h, g = make_integrals(K, seed=0)
    d = DMRG(h, g, K, 0, 64, seed=1, device="cuda", tol=1e-9, max_iter=120, precision=precision)
    d.run(4)
    e_fci = fock.fci_energy(h, g, K, 0)
    for rec in d.log:
        assert rec["energy"] >= e_fci - 1e-10
        if rec["i"] == 3:
            assert abs(rec["energy"] - e_fci) < 1e-10, (rec, e_fci)


def test_thick_restart_converges_to_the_same_eigenpair_in_fewer_steps(device):
    """A small basis (kmax 5) forces many restarts: restarting from [x, previous x]
    reaches the FP64 eigenvalue of the oracle's P^T H P in fewer sigma-vectors
    than restarting from x alone."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.dmrg import Davidson
    from paper_2310_03920_amd.engine import Engine, site_payload
    from paper_2310_03920_amd.mpo import build_nc_mpo
    print("[thick restart]", flush=True)
    K, i = 8, 3
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, 64)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    eng = Engine(build_nc_mpo(h, g), device=device)
    eng.init_boundaries()
    for k in range(i):
        eng.update_left(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], left[k], device))
    for k in range(K - 1, i + 1, -1):
        eng.update_right(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], right[k], device))
    plan = eng.heff_plan(i, bonds[i], bonds[i + 2])
    L, R = eng.left[i], eng.right[i + 2]
    n = int(plan.info.psi_nnz)
    plan.prepare(L, R)
    diag = torch.empty(n, dtype=torch.float64, device=device)
    plan.diag(L, R, diag)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    psi0 = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], np.random.default_rng(5)))).to(device)

    def mv(v, out):
        plan.apply(L, R, v, out)

    e_thin, r_thin, n_thin = Davidson(n, 5, device).solve(mv, psi0, diag, tol=1e-9, max_iter=400, thick=False)
    d = Davidson(n, 5, device)
    e_thick, r_thick, n_thick = d.solve(mv, psi0, diag, tol=1e-9, max_iter=400)
    e_fci = fock.fci_energy(h, g, K, 0)
    print(f"thin {n_thin} matvecs, thick {n_thick} matvecs, E {e_thick:.12f} FCI {e_fci:.12f}", flush=True)
    assert r_thin < 1e-9 and r_thick < 1e-9
    assert abs(e_thick - e_fci) < 1e-10 and abs(e_thin - e_fci) < 1e-10
    assert n_thick < n_thin
    # the returned Ritz vector is normalised and satisfies the residual bound
    hx = torch.empty_like(d.x)
    mv(d.x, hx)
    assert abs(float(d.x.norm()) - 1.0) < 1e-12
    assert float((hx - e_thick * d.x).norm()) < 2e-9


def test_queued_expansion_leaves_the_iterates_unchanged(device):
    """Queueing a step's expansion before its scalars are read (far from convergence)
    gives bitwise the same Ritz value, Ritz vector and sigma-vector count as reading
    them first, through thick restarts (kmax 5)."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.dmrg import Davidson
    from paper_2310_03920_amd.engine import Engine, site_payload
    from paper_2310_03920_amd.mpo import build_nc_mpo
    print("[queued expansion]", flush=True)
    K, i = 8, 3
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, 64)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    eng = Engine(build_nc_mpo(h, g), device=device)
    eng.init_boundaries()
    for k in range(i):
        eng.update_left(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], left[k], device))
    for k in range(K - 1, i + 1, -1):
        eng.update_right(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], right[k], device))
    plan = eng.heff_plan(i, bonds[i], bonds[i + 2])
    L, R = eng.left[i], eng.right[i + 2]
    n = int(plan.info.psi_nnz)
    plan.prepare(L, R)
    diag = torch.empty(n, dtype=torch.float64, device=device)
    plan.diag(L, R, diag)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    psi0 = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], np.random.default_rng(5)))).to(device)

    def mv(v, out):
        plan.apply(L, R, v, out)

    res = {}
    for ahead in (False, True):
        d = Davidson(n, 5, device)
        e, r, nmv = d.solve(mv, psi0, diag, tol=1e-9, max_iter=400, queue_ahead=ahead)
        res[ahead] = (e, r, nmv, d.x.clone())
    assert res[True][:3] == res[False][:3]
    assert torch.equal(res[True][3], res[False][3])
    assert res[True][1] < 1e-9
