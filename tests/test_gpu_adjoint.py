"""GPU parity of the sigma-vector adjoint (hx_heff_apply_backward) with the
oracle's vector-Jacobian products, and autograd energy gradients against
central finite differences.

Tolerance (FP64): each gradient element is a sum of products of the same kind
and length as a sigma element, so the same 1e-11 bound relative to the largest
reference element applies.
"""

import numpy as np
import pytest

from oracle import contract, mps
from synth.blocks import random_env, random_psi, two_site_blocks
from test_gpu_parity import _problem

pytestmark = pytest.mark.gpu

RTOL = 1e-11


def _rel(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _oracle_vjp(X, lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi, g):
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    Ld, Rd = contract.dense_env(L, lb), contract.dense_env(R, rb)
    D1, D2 = contract.dense_mpo(W1, len(Ldq), len(Mdq)), contract.dense_mpo(W2, len(Mdq), len(Rdq))
    rL, rW1, rW2, rR, rpsi = contract.heff_vjp(Ld, D1, D2, Rd, mps.dense_two_site(psi, lb, rb),
                                               mps.dense_two_site(g, lb, rb))
    return {
        "psi": X.pack_psi(lbB, rbB, mps.two_site_blocks_from_dense(rpsi, lb, rb, two_site_blocks(lb, rb))),
        "L": X.pack_env(lbB, Ldq, contract.env_blocks_from_dense(rL, lb, Ldq)),
        "R": X.pack_env(rbB, Rdq, contract.env_blocks_from_dense(rR, rb, Rdq)),
        "W1": np.array([np.where(op != 0, rW1[a, b], 0).ravel() for a, b, op in W1]).ravel(),
        "W2": np.array([np.where(op != 0, rW2[b, c], 0).ravel() for b, c, op in W2]).ravel(),
    }


def _gpu_vjp(device, X, lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi, g, **opts):
    import torch
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffVjpPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, **opts).upload(device)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    Lt, Rt = t(X.pack_env(lbB, Ldq, L)), t(X.pack_env(rbB, Rdq, R))
    pt, gt = t(X.pack_psi(lbB, rbB, psi)), t(X.pack_psi(lbB, rbB, g))
    out = {k: torch.full((n,), float("nan"), dtype=torch.float64, device=device)
           for k, n in (("psi", pt.numel()), ("L", Lt.numel()), ("R", Rt.numel()),
                        ("W1", 16 * len(W1)), ("W2", 16 * len(W2)))}
    plan.prepare(Lt, Rt)
    plan.backward(Lt, Rt, pt, gt, out["psi"], out["L"], out["R"], out["W1"], out["W2"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, plan


@pytest.mark.parametrize("seed,big,opts", [(0, False, {}), (1, True, {}), (3, True, {"split_kseg_min": 16}),
                                           (6, True, {"t_budget_bytes": 256 * 1024}),
                                           (4, True, {"kernel_variant": 1}), (5, True, {"kernel_variant": 2}),
                                           (7, True, {"kernel_variant": 4}), (8, True, {"kernel_variant": 5})])
def test_backward_matches_oracle(device, seed, big, opts):
    from paper_2310_03920_amd import _lib as X
    print(f"[heff_apply_backward] seed={seed} big={big} opts={opts}", flush=True)
    prob = _problem(seed, big)
    g = random_psi(prob[0], prob[1], np.random.default_rng(50 + seed))
    got, plan = _gpu_vjp(device, X, *prob, g, **opts)
    if "t_budget_bytes" in opts:
        assert plan.info.n_chunks > 2
    ref = _oracle_vjp(X, *prob, g)
    for k in ref:
        assert _rel(got[k], ref[k]) <= RTOL, (k, _rel(got[k], ref[k]))


def test_backward_real_mpo_all_sites(device):
    """NC-partition MPO (aliased and shared mixed operators) at every site pair of a
    6-orbital chain."""
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    from synth import bond_sector_tables, make_integrals
    K = 6
    m = build_nc_mpo(*make_integrals(K, seed=3))
    b = bond_sector_tables(K, K, 0, 12, model="gaussian")
    for i in range(K - 1):
        print(f"[heff_apply_backward] real MPO K=6 site {i}", flush=True)
        rng = np.random.default_rng(i)
        lb, rb = b[i], b[i + 2]
        Ldq, Mdq, Rdq = ([tuple(x) for x in m.dq[k]] for k in (i, i + 1, i + 2))
        prob = (lb, rb, Ldq, Mdq, Rdq, random_env(lb, Ldq, rng), random_env(rb, Rdq, rng),
                site_entries(m, i), site_entries(m, i + 1), random_psi(lb, rb, rng))
        g = random_psi(lb, rb, rng)
        got, _ = _gpu_vjp(device, X, *prob, g)
        ref = _oracle_vjp(X, *prob, g)
        for k in ref:
            assert _rel(got[k], ref[k]) <= RTOL, (i, k, _rel(got[k], ref[k]))


def test_backward_is_bitwise_repeatable(device):
    from paper_2310_03920_amd import _lib as X
    print("[heff_apply_backward repeat]", flush=True)
    prob = _problem(2, True)
    g = random_psi(prob[0], prob[1], np.random.default_rng(7))
    a, _ = _gpu_vjp(device, X, *prob, g)
    b, _ = _gpu_vjp(device, X, *prob, g)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_autograd_energy_gradient_matches_central_differences(device):
    """E = <psi| H_eff |psi> through torch.autograd; its gradient along random
    directions of psi, L, R, W1 and W2 against central differences (step 1e-5) of
    the GPU forward pass, to 1e-6 relative."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.autograd import HeffOperator
    print("[autograd] energy gradient vs central differences", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(1, True)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    op = HeffOperator(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, device=device)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    Lt = t(X.pack_env(lbB, Ldq, L)).requires_grad_()
    Rt = t(X.pack_env(rbB, Rdq, R)).requires_grad_()
    pt = t(X.pack_psi(lbB, rbB, psi))
    pt = (pt / pt.norm()).requires_grad_()
    w1, w2 = (w.requires_grad_() for w in op.values())
    E = torch.dot(pt, op(Lt, Rt, w1, w2, pt))
    grads = torch.autograd.grad(E, [pt, Lt, Rt, w1, w2])

    def energy(psi_, L_, R_, W1_=W1, W2_=W2):
        o = op if (W1_ is W1 and W2_ is W2) else HeffOperator(lbB, rbB, Ldq, Mdq, Rdq, W1_, W2_, device=device)
        with torch.no_grad():
            a, b = o.values()
            return float(torch.dot(psi_, o(L_, R_, a, b, psi_)))

    rng = np.random.default_rng(3)
    h = 1e-5
    base = [pt.detach(), Lt.detach(), Rt.detach()]
    for slot in range(3):
        V = t(rng.standard_normal(base[slot].numel()))
        ap, am = list(base), list(base)
        ap[slot] = base[slot] + h * V
        am[slot] = base[slot] - h * V
        fd = (energy(*ap) - energy(*am)) / (2 * h)
        an = float(torch.dot(grads[slot], V))
        assert an == pytest.approx(fd, rel=1e-6), (slot, an, fd)
    for slot, W in ((3, W1), (4, W2)):
        V = [rng.standard_normal((4, 4)) * (op_ != 0) for _, _, op_ in W]
        Wp = [(a, b, op_ + h * v) for (a, b, op_), v in zip(W, V)]
        Wm = [(a, b, op_ - h * v) for (a, b, op_), v in zip(W, V)]
        args = (base[0], base[1], base[2])
        fd = ((energy(*args, Wp, W2) if slot == 3 else energy(*args, W1, Wp)) -
              (energy(*args, Wm, W2) if slot == 3 else energy(*args, W1, Wm))) / (2 * h)
        an = float((grads[slot].cpu() * torch.from_numpy(np.array(V))).sum())
        assert an == pytest.approx(fd, rel=1e-6), (slot, an, fd)


@pytest.mark.parametrize("seed,opts", [(1, {}), (6, {"t_budget_bytes": 256 * 1024, "kernel_variant": 1})])
def test_backward_f32_matches_oracle_to_fp32_accuracy(device, seed, opts):
    """FP32 operands and accumulation (hx_heff_apply_backward_f32): every gradient
    within 2e-4 of the oracle's FP64 value, relative to its largest entry (inputs
    rounded once to 2^-24, FP32 sums over <= ~2e3 terms), same as the FP32 sigma."""
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[backward f32] seed={seed} {opts}", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(seed, True)
    rng = np.random.default_rng(70 + seed)
    g = random_psi(lb, rb, rng)
    ref = _oracle_vjp(X, lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi, g)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffVjpPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, **opts).upload(device)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    Lt, Rt = t(X.pack_env(lbB, Ldq, L)), t(X.pack_env(rbB, Rdq, R))
    p32 = t(X.pack_psi(lbB, rbB, psi)).float()
    g32 = t(X.pack_psi(lbB, rbB, g)).float()
    plan.prepare(Lt, Rt)
    plan.lower_f32(Lt, Rt)
    out = {k: torch.full((n,), float("nan"), dtype=torch.float32, device=device)
           for k, n in (("psi", p32.numel()), ("L", Lt.numel()), ("R", Rt.numel()),
                        ("W1", 16 * len(W1)), ("W2", 16 * len(W2)))}
    plan.backward_f32(p32, g32, out["psi"], out["L"], out["R"], out["W1"], out["W2"])
    torch.cuda.synchronize()
    for k in ref:
        err = _rel(out[k].double().cpu().numpy(), ref[k])
        print(f"  {k}: rel err {err:.2e}", flush=True)
        assert err <= 2e-4, (k, err)
