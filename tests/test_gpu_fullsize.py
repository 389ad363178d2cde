"""Parity at the benchmark's full size.

The middle site pair (17, 18) of the 36-orbital chain at M = 1000 (NC MPO,
Gaussian sector model of width 1, integrals seed 0), with seeded N(0,1)
environments and psi, is applied with the plan options the benchmark's autotuner
chooses for it (kernel variant 1, split-K segments of 512, intermediate budget 1 or
2 GiB).  Sampled rows of sigma -- the first and last rows of the largest left
sector (the last one in a ragged 64-row tile), a row of the smallest sector
and random rows -- are compared with the oracle, which computes each row on its
own straight from the block formats.
"""

import numpy as np
import pytest

from oracle import contract
from synth import bond_sector_tables, make_integrals
from synth.blocks import random_env, random_psi

pytestmark = pytest.mark.gpu

K, M = 36, 1000
SITE = K // 2 - 1


@pytest.fixture(scope="module")
def problem(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    print(f"[full size] building {K} orbitals, M={M}, sites ({SITE}, {SITE + 1})", flush=True)
    mpo = build_nc_mpo(*make_integrals(K, seed=0))
    bonds = bond_sector_tables(K, K, 0, M, model="gaussian", width=1.0)
    lb, rb = bonds[SITE], bonds[SITE + 2]
    rng = np.random.default_rng(2024)
    Ldq = [tuple(x) for x in mpo.dq[SITE]]
    Rdq = [tuple(x) for x in mpo.dq[SITE + 2]]
    L = random_env(lb, Ldq, rng)
    R = random_env(rb, Rdq, rng)
    psi = random_psi(lb, rb, rng)
    W1, W2 = site_entries(mpo, SITE), site_entries(mpo, SITE + 1)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    dev = dict(
        L=torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device),
        R=torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device),
        psi=torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device),
    )
    # sampled rows (il', s1', x)
    big = max(range(len(lb)), key=lambda j: lb[j][1])
    one = min(range(len(lb)), key=lambda j: lb[j][1])
    rows = [(big, 1, 0), (big, 2, lb[big][1] - 1), (one, 0, 0)]
    pick = np.random.default_rng(5)
    while len(rows) < 6:
        il = int(pick.integers(len(lb)))
        rows.append((il, int(pick.integers(4)), int(pick.integers(lb[il][1]))))
    print(f"[full size] oracle rows {rows}", flush=True)
    ref = contract.sigma_rows(lb, rb, L, W1, W2, R, psi, rows)
    W1s = X.MpoSite(mpo.sites[SITE].rows, mpo.sites[SITE].cols, mpo.sites[SITE].mats)
    W2s = X.MpoSite(mpo.sites[SITE + 1].rows, mpo.sites[SITE + 1].cols, mpo.sites[SITE + 1].mats)
    return dict(lb=lb, rb=rb, lbB=lbB, rbB=rbB, Ldq=Ldq, Rdq=Rdq, mpo=mpo, W1=W1s, W2=W2s, dev=dev,
                rows=rows, ref=ref)


@pytest.mark.parametrize("budget_gb,variant", [(2.0, 1), (1.0, 1)])
def test_fullsize_sigma_rows_match_the_oracle(device, problem, budget_gb, variant):
    import torch
    from paper_2310_03920_amd import _lib as X
    p = problem
    print(f"[full size] apply, variant {variant}, kseg 512, budget {budget_gb} GiB", flush=True)
    mid = [tuple(x) for x in p["mpo"].dq[SITE + 1]]
    plan = X.HeffPlan(p["lbB"], p["rbB"], p["Ldq"], mid, p["Rdq"], p["W1"], p["W2"],
                      t_budget_bytes=int(budget_gb * (1 << 30)), split_kseg_min=512,
                      kernel_variant=variant).upload(device)
    d = p["dev"]
    plan.prepare(d["L"], d["R"])
    sigma = torch.full_like(d["psi"], float("nan"))
    plan.apply(d["L"], d["R"], d["psi"], sigma)
    torch.cuda.synchronize()
    got = X.unpack_psi(p["lbB"], p["rbB"], sigma.cpu().numpy())
    scale = max(float(np.max(np.abs(v))) for r in p["ref"].values() for v in r.values())
    worst = 0.0
    for (il, s1, x), cols in p["ref"].items():
        for (s2, ir), vec in cols.items():
            g = got[(il, s1, s2, ir)][x]
            worst = max(worst, float(np.max(np.abs(g - vec))))
    print(f"[full size] max |gpu - oracle| = {worst:.3e} (scale {scale:.3e})", flush=True)
    assert worst <= 1e-11 * scale
    del plan


@pytest.mark.parametrize("mode,rtol", [("f32", 2e-4), ("bf16", 2e-2)])
def test_fullsize_reduced_precision_sigma_rows_match_the_oracle(device, problem, mode, rtol):
    """FP32 and BF16 block products (FP32 accumulation) at the benchmark shape and
    launch configuration, against the FP64 oracle's rows: FP32 operands carry 2^-24
    relative rounding, BF16 ones 2^-9 (operands and the stage-1 intermediate), with
    FP32 accumulation over sums of up to ~10^4 products of random sign."""
    import torch
    from paper_2310_03920_amd import _lib as X
    p = problem
    print(f"[full size] {mode} apply, variant 1, kseg 512, budget 1 GiB", flush=True)
    mid = [tuple(x) for x in p["mpo"].dq[SITE + 1]]
    plan = X.HeffPlan(p["lbB"], p["rbB"], p["Ldq"], mid, p["Rdq"], p["W1"], p["W2"],
                      t_budget_bytes=1 << 30, split_kseg_min=512, kernel_variant=1).upload(device)
    d = p["dev"]
    plan.prepare(d["L"], d["R"])
    plan.lower_f32(d["L"], d["R"])
    psi32 = d["psi"].float()
    sig32 = torch.full_like(psi32, float("nan"))
    (plan.apply_bf16 if mode == "bf16" else plan.apply_f32)(psi32, sig32)
    torch.cuda.synchronize()
    got = X.unpack_psi(p["lbB"], p["rbB"], sig32.double().cpu().numpy())
    scale = max(float(np.max(np.abs(v))) for r in p["ref"].values() for v in r.values())
    worst = max(float(np.max(np.abs(got[(il, s1, s2, ir)][x] - vec)))
                for (il, s1, x), cols in p["ref"].items() for (s2, ir), vec in cols.items())
    print(f"[full size] {mode}: max |gpu - oracle| = {worst:.3e} (scale {scale:.3e}, ratio {worst / scale:.2e})",
          flush=True)
    assert worst <= rtol * scale
    del plan


def test_fullsize_environment_update_rows_match_the_oracle(device):
    """The left environment update at the benchmark's middle site (site 17 of the
    36-orbital chain, M = 1000, NC MPO: 2424 -> 2702 operators) with a seeded N(0,1)
    environment and a seeded left-canonical site tensor, in the launch configuration
    of the sweep engine, against the oracle's rows of L'_b by definition."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.engine import Engine
    from paper_2310_03920_amd.mpo import build_nc_mpo, site_entries
    from synth import random_left_canonical_mps
    print("[full size] env update rows, 36 orbitals, M=1000, site 17", flush=True)
    mpo = build_nc_mpo(*make_integrals(K, seed=0))
    bonds = bond_sector_tables(K, K, 0, M, model="gaussian", width=1.0)
    k = SITE
    bi, bo = bonds[k], bonds[k + 1]
    dqi, dqo = [tuple(x) for x in mpo.dq[k]], [tuple(x) for x in mpo.dq[k + 1]]
    rng = np.random.default_rng(77)
    Lenv = random_env(bi, dqi, rng)
    A = random_left_canonical_mps(bonds, 3)[k]
    biB, boB = X.Bond(bi), X.Bond(bo)
    plan = X.EnvPlan(0, biB, boB, dqi, dqo, X.MpoSite(mpo.sites[k].rows, mpo.sites[k].cols, mpo.sites[k].mats),
                     **Engine.PLAN_OPTS).upload(device)
    Lt = torch.from_numpy(X.pack_env(biB, dqi, Lenv)).to(device)
    At = torch.from_numpy(X.pack_site(biB, boB, A)).to(device)
    out = torch.full((int(plan.info.out_nnz),), float("nan"), dtype=torch.float64, device=device)
    plan.update(Lt, At, out)
    torch.cuda.synchronize()
    flat = out.cpu().numpy()
    assert np.isfinite(flat).all()
    op_off, blk_off = X.env_layout(boB, X.OpSet(dqo))
    idx = {q: j for j, (q, _) in enumerate(bo)}
    pick = np.random.default_rng(8)
    rows = []
    for b in (0, len(dqo) // 2, len(dqo) - 1, int(pick.integers(len(dqo)))):
        dq = dqo[b]
        dsts = [idx[(q[0] + dq[0], q[1] + dq[1])] for q, _ in bo if (q[0] + dq[0], q[1] + dq[1]) in idx]
        iq = max(dsts, key=lambda j: bo[j][1])
        rows += [(b, iq, 0), (b, iq, bo[iq][1] - 1)]
    ref = contract.env_rows_left(bi, bo, Lenv, site_entries(mpo, k), A, rows)
    worst, scale = 0.0, 0.0
    for (b, iq, m), acc in ref.items():
        for iqn, vec in acc.items():
            o = int(blk_off[b, iqn])
            g = flat[o + m * bo[iqn][1]:o + (m + 1) * bo[iqn][1]]
            worst = max(worst, float(np.max(np.abs(g - vec))))
            scale = max(scale, float(np.max(np.abs(vec))))
    print(f"[full size] env rows {len(rows)}: max |gpu - oracle| = {worst:.3e} (scale {scale:.3e})", flush=True)
    assert scale > 0 and worst <= 1e-11 * scale


def _big_case(device, K_, M_, budget_gib, modes):
    import time
    import torch
    from paper_2310_03920_amd import _lib as X
    from fullsize_data import compare_rows, middle_problem, sample_rows
    t0 = time.time()
    p = middle_problem(X, K_, M_)
    rows = sample_rows(p["lb"], 4)
    print(f"[full size] {K_} orbitals M={M_}: operands drawn in {time.time() - t0:.0f}s; oracle rows {rows}",
          flush=True)
    t0 = time.time()
    ref = contract.sigma_rows(p["bonds"][p["i"]], p["bonds"][p["i"] + 2], p["L"], p["W1e"], p["W2e"], p["R"],
                              p["psi"], rows)
    print(f"[full size] oracle rows in {time.time() - t0:.0f}s", flush=True)
    plan = X.HeffPlan(p["lb"], p["rb"], p["Ldq"], p["Mdq"], p["Rdq"], p["W1"], p["W2"],
                      t_budget_bytes=int(budget_gib * (1 << 30)), split_kseg_min=512,
                      kernel_variant=1).upload(device)
    print(f"[full size] plan: {plan.info.n_chunks} chunks, {plan.info.flops_useful / 1e12:.2f} TFLOP", flush=True)
    L = torch.from_numpy(p["Lf"]).to(device)
    R = torch.from_numpy(p["Rf"]).to(device)
    psi = torch.from_numpy(p["Pf"]).to(device)
    plan.prepare(L, R)
    res = {}
    for mode in modes:
        if mode == "f64":
            sig = torch.full_like(psi, float("nan"))
            plan.apply(L, R, psi, sig)
            host = sig.cpu().numpy()
        else:
            if getattr(plan, "L32", None) is None:
                plan.lower_f32(L, R)
            s32 = torch.full_like(psi, float("nan"), dtype=torch.float32)
            (plan.apply_bf16 if mode == "bf16" else plan.apply_f32)(psi.float(), s32)
            host = s32.double().cpu().numpy()
        torch.cuda.synchronize()
        res[mode] = compare_rows(X, p["lb"], p["rb"], host, ref)
        print(f"[full size] {K_}/{M_} {mode}: max |gpu - oracle| = {res[mode][0]:.3e} (scale {res[mode][1]:.3e})",
              flush=True)
    return res


def test_fullsize_48_orbitals_m2000_sigma_rows_match_the_oracle(device):
    """The batched-mode configuration's large instance: the middle of the 48-orbital
    chain at M = 2000 (blocks up to 248 rows, MPO bond dimensions 4380 / 4754 / 5144,
    26 intermediate chunks at a 4 GiB budget) in the profiled launch configuration,
    FP64 / FP32 / BF16 block products against the oracle's rows."""
    res = _big_case(device, 48, 2000, 4.0, ("f64", "f32", "bf16"))
    for mode, tol in (("f64", 1e-11), ("f32", 2e-4), ("bf16", 2e-2)):
        worst, scale = res[mode]
        assert scale > 0 and worst <= tol * scale, mode


def test_fullsize_36_orbitals_m2000_sigma_rows_match_the_oracle(device):
    """The precision-mode configuration at its larger bond dimension (36 orbitals,
    M = 2000, 2 GiB intermediate budget), FP64 against the oracle's rows."""
    res = _big_case(device, 36, 2000, 2.0, ("f64",))
    worst, scale = res["f64"]
    assert scale > 0 and worst <= 1e-11 * scale


def test_backward_at_config5_size_satisfies_euler_identities(device):
    """Adjoint at the middle of the 24-orbital chain, M = 500 (NC MPO, seeded N(0,1)
    environments, psi and cotangent g).  sigma is linear in each of psi, L, R, W1,
    W2 separately, so <g_X, X> = <g, sigma> for every one of them -- identities
    that hold at any size and fail for a dropped, duplicated or misplaced term."""
    import time
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.mpo import build_nc_mpo
    K2, M2 = 24, 500
    i = K2 // 2 - 1
    print(f"[full size] backward, {K2} orbitals, M={M2}", flush=True)
    mpo = build_nc_mpo(*make_integrals(K2, seed=0))
    bonds = bond_sector_tables(K2, K2, 0, M2, model="gaussian", width=1.0)
    lb, rb = bonds[i], bonds[i + 2]
    rng = np.random.default_rng(11)
    Ldq = [tuple(x) for x in mpo.dq[i]]
    Mdq = [tuple(x) for x in mpo.dq[i + 1]]
    Rdq = [tuple(x) for x in mpo.dq[i + 2]]
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    W1 = X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats)
    W2 = X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats)
    opts = dict(kernel_variant=1, split_kseg_min=512)
    fwd = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, **opts).upload(device)
    vjp = X.HeffVjpPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, **opts).upload(device)
    f64 = dict(dtype=torch.float64, device=device)
    L = torch.from_numpy(X.pack_env(lbB, Ldq, random_env(lb, Ldq, rng))).to(device)
    R = torch.from_numpy(X.pack_env(rbB, Rdq, random_env(rb, Rdq, rng))).to(device)
    psi = torch.from_numpy(X.pack_psi(lbB, rbB, random_psi(lb, rb, rng))).to(device)
    g = torch.from_numpy(X.pack_psi(lbB, rbB, random_psi(lb, rb, rng))).to(device)
    sigma = torch.empty_like(psi)
    fwd.prepare(L, R)
    fwd.apply(L, R, psi, sigma)
    g_psi, g_L, g_R = torch.empty_like(psi), torch.empty_like(L), torch.empty_like(R)
    g_w1 = torch.empty(16 * vjp.nnz1, **f64)
    g_w2 = torch.empty(16 * vjp.nnz2, **f64)
    vjp.prepare(L, R)
    torch.cuda.synchronize()
    t = time.perf_counter()
    vjp.backward(L, R, psi, g, g_psi, g_L, g_R, g_w1, g_w2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ref = float(torch.dot(g, sigma))
    w1 = torch.from_numpy(W1.vals.ravel().copy()).to(device)
    w2 = torch.from_numpy(W2.vals.ravel().copy()).to(device)
    got = {"psi": float(torch.dot(g_psi, psi)), "L": float(torch.dot(g_L, L)), "R": float(torch.dot(g_R, R)),
           "W1": float(torch.dot(g_w1, w1)), "W2": float(torch.dot(g_w2, w2))}
    print(f"[full size] backward {1e3 * dt:.1f} ms ({vjp.info.flops_apply / 1e12:.3f} TFLOP); <g, sigma> = {ref:.12e}; "
          + ", ".join(f"{k}: {v:.12e}" for k, v in got.items()), flush=True)
    for k, v in got.items():
        assert abs(v - ref) <= 1e-11 * (abs(ref) + float(torch.linalg.vector_norm(g)) *
                                         float(torch.linalg.vector_norm(sigma))), k
