"""Batched sigma-vectors (several independent two-site problems per launch) and
HIP-graph replay of the launch sequence, on the GPU.

A batched plan runs the same tiles with the same task order as each instance's
own plan, so every instance's output must equal its own plan's output bit for
bit; one instance is also checked against the FP64 oracle.
"""

import numpy as np
import pytest

from test_gpu_parity import _close, _dense_sigma, _problem

pytestmark = pytest.mark.gpu

CASES = [(0, False, 0), (1, True, 0), (2, False, 8), (3, True, 16), (4, True, 0)]


def _instances(device, cases=CASES, variant=0, budget=None):
    import torch
    from paper_2310_03920_amd import _lib as X
    out = []
    extra = {} if budget is None else {"t_budget_bytes": budget}
    for seed, big, kseg in cases:
        prob = _problem(seed, big)
        lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob
        lbB, rbB = X.Bond(lb), X.Bond(rb)
        plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, split_kseg_min=kseg, kernel_variant=variant, **extra)
        arrs = (X.pack_env(lbB, Ldq, L), X.pack_env(rbB, Rdq, R), X.pack_psi(lbB, rbB, psi))
        out.append((prob, plan, arrs))
    return out


def _concat(B, insts, device):
    import torch
    Ls = [torch.from_numpy(a[0]) for _, _, a in insts]
    Rs = [torch.from_numpy(a[1]) for _, _, a in insts]
    Ps = [torch.from_numpy(a[2]) for _, _, a in insts]
    for i, (po, lo, ro) in enumerate(B.offsets):
        assert po == sum(p.numel() for p in Ps[:i]) and lo == sum(x.numel() for x in Ls[:i])
        assert ro == sum(x.numel() for x in Rs[:i])
    return (torch.cat(Ls).to(device), torch.cat(Rs).to(device), torch.cat(Ps).to(device))


def _individual(device, plan, arrs, f32=False):
    import torch
    plan.upload(device)
    L, R, p = (torch.from_numpy(a).to(device) for a in arrs)
    plan.prepare(L, R)
    s = torch.full_like(p, float("nan"))
    plan.apply(L, R, p, s)
    d = torch.full_like(p, float("nan"))
    plan.diag(L, R, d)
    res = {"sigma": s.cpu(), "diag": d.cpu()}
    if f32:
        plan.lower_f32(L, R)
        p32 = p.float()
        s32 = torch.full_like(p32, float("nan"))
        plan.apply_f32(p32, s32)
        res["sigma32"] = s32.cpu()
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("variant,budget", [(0, None), (5, None), (6, None), (1, 96 * 1024)])
def test_batched_apply_and_diag_match_instances_bitwise(device, variant, budget):
    """Each instance of a batched plan gives, bit for bit, its own plan's sigma and
    diag, in FP64 and FP32, for the two-buffer, tile-shape and single-wave kernels,
    and for instances split into several intermediate chunks (merged round by round)."""
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[batch] 5 instances, f64 + f32, variant {variant}, budget {budget}", flush=True)
    insts = _instances(device, variant=variant, budget=budget)
    if budget is not None:
        chunks = [plan.info.n_chunks for _, plan, _ in insts]
        assert max(chunks) > 2 and len(set(chunks)) > 1, chunks
    ref = [_individual(device, plan, arrs, f32=True) for _, plan, arrs in insts]
    B = X.BatchPlan([plan for _, plan, _ in insts]).upload(device)
    assert B.info.flops_apply == pytest.approx(sum(p.info.flops_apply for _, p, _ in insts), rel=1e-12)
    L, R, p = _concat(B, insts, device)
    B.prepare(L, R)
    s = torch.full_like(p, float("nan"))
    B.apply(L, R, p, s)
    d = torch.full_like(p, float("nan"))
    B.diag(L, R, d)
    B.lower_f32(L, R)
    p32 = p.float()
    s32 = torch.full_like(p32, float("nan"))
    B.apply_f32(p32, s32)
    torch.cuda.synchronize()
    s, d, s32 = s.cpu(), d.cpu(), s32.cpu()
    for i, (po, _, _) in enumerate(B.offsets):
        n = ref[i]["sigma"].numel()
        assert torch.equal(s[po:po + n], ref[i]["sigma"]), i
        assert torch.equal(d[po:po + n], ref[i]["diag"]), i
        assert torch.equal(s32[po:po + n], ref[i]["sigma32"]), i
    prob, plan, _ = insts[1]
    lbB, rbB = X.Bond(prob[0]), X.Bond(prob[1])
    po = B.offsets[1][0]
    _close(X.unpack_psi(lbB, rbB, s[po:po + ref[1]["sigma"].numel()].numpy()), _dense_sigma(*prob))


def test_graph_replays_match_eager(device):
    """Replays of a captured prepare+apply sequence, with eager work and new
    psi contents between them, each equal the eager result bit for bit."""
    import torch
    from paper_2310_03920_amd import _lib as X
    print("[graph] batched prepare+apply, 3 replays", flush=True)
    insts = _instances(device, CASES[:3])
    B = X.BatchPlan([plan for _, plan, _ in insts]).upload(device)
    L, R, p = _concat(B, insts, device)
    s_graph = torch.full_like(p, float("nan"))
    g = X.Graph(B, X.GRAPH_PREPARE_APPLY, L, R, B.ws, p, s_graph)
    s_eager = torch.empty_like(p)
    gen = torch.Generator(device="cpu").manual_seed(7)
    for rep in range(3):
        if rep:
            p.copy_(torch.randn(p.numel(), generator=gen, dtype=torch.float64).to(device))
        s_graph.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        got = s_graph.clone()
        B.prepare(L, R)
        B.apply(L, R, p, s_eager)
        junk = (s_eager * 2.0).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(got, s_eager), rep
    del g


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_graph_f32_apply_replays(device, mode):
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[graph] single-plan {mode} apply", flush=True)
    (prob, plan, arrs), = _instances(device, CASES[1:2])
    plan.upload(device)
    L, R, p = (torch.from_numpy(a).to(device) for a in arrs)
    plan.prepare(L, R)
    plan.lower_f32(L, R)
    p32 = p.float()
    s_graph = torch.full_like(p32, float("nan"))
    what = X.GRAPH_APPLY_BF16 if mode == "bf16" else X.GRAPH_APPLY_F32
    g = X.Graph(plan, what, plan.L32, plan.R32, plan.ws32, p32, s_graph)
    s_eager = torch.empty_like(p32)
    (plan.apply_bf16 if mode == "bf16" else plan.apply_f32)(p32, s_eager)
    for rep in range(2):
        s_graph.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(s_graph, s_eager), rep


def test_batched_real_mpo_instances(device):
    """Instances of the ab initio NC MPO with different centres and electron
    numbers (the mixed-size batch), batched vs one by one."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    from synth import bond_sector_tables, make_integrals
    from synth.blocks import random_env, random_psi
    print("[batch] real MPO K=10 mixed N / centre", flush=True)
    K = 10
    insts = []
    for j, (N, i) in enumerate([(8, 2), (10, 4), (12, 6), (10, 3)]):
        rng = np.random.default_rng(100 + j)
        m = build_nc_mpo(*make_integrals(K, seed=j + 1))
        b = bond_sector_tables(K, N, 0, 48, model="gaussian")
        lb, rb = b[i], b[i + 2]
        Ldq, Rdq = [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]]
        lbB, rbB = X.Bond(lb), X.Bond(rb)
        plan = X.HeffPlan(lbB, rbB, m.dq[i], m.dq[i + 1], m.dq[i + 2], site_entries(m, i), site_entries(m, i + 1))
        arrs = (X.pack_env(lbB, Ldq, random_env(lb, Ldq, rng)), X.pack_env(rbB, Rdq, random_env(rb, Rdq, rng)),
                X.pack_psi(lbB, rbB, random_psi(lb, rb, rng)))
        insts.append((None, plan, arrs))
    ref = [_individual(device, plan, arrs) for _, plan, arrs in insts]
    B = X.BatchPlan([plan for _, plan, _ in insts]).upload(device)
    L, R, p = _concat(B, insts, device)
    B.prepare(L, R)
    s = torch.full_like(p, float("nan"))
    B.apply(L, R, p, s)
    torch.cuda.synchronize()
    s = s.cpu()
    for i, (po, _, _) in enumerate(B.offsets):
        n = ref[i]["sigma"].numel()
        assert torch.equal(s[po:po + n], ref[i]["sigma"]), i
