"""GPU parity of the HIP path against the FP64 oracle, element by element.

Tolerance (FP64): every output is a sum of at most ~1e4 products formed and
accumulated in IEEE double; the accumulated rounding is bounded by
n * 2^-53 * sum|terms| <~ 1e-12 of the largest output here, so elements must
agree to 1e-11 relative to the largest reference element.
"""

import numpy as np
import pytest

from oracle import contract, davidson, mps
from synth import bond_sector_tables, make_integrals, random_left_canonical_mps, random_right_canonical_mps
from synth.blocks import random_env, random_psi, random_site_ops, random_site_tensor, two_site_blocks

pytestmark = pytest.mark.gpu

RTOL = 1e-11

DQS = [(0, 0), (1, 1), (1, -1), (-1, 1), (-1, -1), (0, 2), (0, -2), (2, 0), (-2, 0)]


def _bonds(seed, big):
    rng = np.random.default_rng(seed)
    lq = [(2, -2), (2, 0), (2, 2), (3, -1), (3, 1), (4, 0)]
    rq = [(3, -1), (3, 1), (4, -2), (4, 0), (4, 2), (5, -1), (5, 1), (6, 0)]
    dims = [1, 3, 17, 64, 65, 130] if big else [1, 2, 5, 9]
    lb = [(q, int(rng.choice(dims))) for q in lq]
    rb = [(q, int(rng.choice(dims))) for q in rq]
    return lb, rb


def _problem(seed, big=False, nL=7, nM=9, nR=7):
    rng = np.random.default_rng(seed)
    lb, rb = _bonds(seed, big)
    Ldq = [DQS[i % len(DQS)] for i in range(nL)]
    Mdq = [DQS[(i * 5) % len(DQS)] for i in range(nM)]
    Rdq = [DQS[(i * 7 + 3) % len(DQS)] for i in range(nR)]
    L = random_env(lb, Ldq, rng)
    R = random_env(rb, Rdq, rng)
    W1 = random_site_ops(Ldq, Mdq, rng, per_col=3)
    W2 = random_site_ops(Mdq, Rdq, rng, per_col=3)
    psi = random_psi(lb, rb, rng)
    return lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi


def _dense_sigma(lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi):
    s = contract.heff_apply(contract.dense_env(L, lb), contract.dense_mpo(W1, len(Ldq), len(Mdq)),
                            contract.dense_mpo(W2, len(Mdq), len(Rdq)), contract.dense_env(R, rb),
                            mps.dense_two_site(psi, lb, rb))
    return mps.two_site_blocks_from_dense(s, lb, rb, two_site_blocks(lb, rb))


def _close(got, ref, rtol=RTOL):
    scale = max(max(np.abs(v).max() for v in ref.values() if v.size), 1e-300)
    for k in ref:
        err = np.abs(got[k] - ref[k]).max() if ref[k].size else 0.0
        assert err <= rtol * scale, (k, err, scale)


def _run_heff(device, lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi, budget=0, diag=False, kseg=0, variant=0,
              merge_off=0):
    import torch
    from paper_2310_03920_amd import _lib as X
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, t_budget_bytes=budget,
                      split_kseg_min=kseg, kernel_variant=variant, t_merge_off=merge_off).upload(device)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    st = torch.full_like(pt, float("nan"))
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pt, st)
    out = {"sigma": X.unpack_psi(lbB, rbB, st.cpu().numpy()), "plan": plan}
    if diag:
        dt = torch.full_like(pt, float("nan"))
        plan.diag(Lt, Rt, dt)
        out["diag"] = X.unpack_psi(lbB, rbB, dt.cpu().numpy())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("seed,big", [(0, False), (1, True), (2, True)])
def test_heff_apply_random_operands(device, seed, big):
    print(f"[heff_apply] seed={seed} big={big}", flush=True)
    prob = _problem(seed, big)
    got = _run_heff(device, *prob)["sigma"]
    _close(got, _dense_sigma(*prob))


def test_heff_apply_chunked_intermediates(device):
    print("[heff_apply chunked]", flush=True)
    prob = _problem(3, True)
    res = _run_heff(device, *prob, budget=256 * 1024)
    assert res["plan"].info.n_chunks > 2
    _close(res["sigma"], _dense_sigma(*prob))


@pytest.mark.parametrize("kseg", [8, 33])
def test_heff_apply_split_k(device, kseg):
    """Long task lists cut into split-K segments summed by the fixed-order reduction."""
    print(f"[heff_apply split-K] kseg={kseg}", flush=True)
    prob = _problem(6, True)
    res = _run_heff(device, *prob, kseg=kseg, budget=512 * 1024)
    _close(res["sigma"], _dense_sigma(*prob))


@pytest.mark.parametrize("variant", [1, 2, 4, 5, 6])
def test_heff_apply_kernel_variants(device, variant):
    """One-buffer and 8-deep pipelines: same results as the oracle, incl. split-K and diag."""
    print(f"[heff_apply variant] {variant}", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob = _problem(2, True)
    res = _run_heff(device, *prob, kseg=16, variant=variant, diag=True)
    _close(res["sigma"], _dense_sigma(*prob))
    d = contract.heff_diag(contract.dense_env(L, lb), contract.dense_mpo(W1, len(Ldq), len(Mdq)),
                           contract.dense_mpo(W2, len(Mdq), len(Rdq)), contract.dense_env(R, rb))
    _close(res["diag"], mps.two_site_blocks_from_dense(d, lb, rb, two_site_blocks(lb, rb)))


@pytest.mark.parametrize("merge_off,budget", [(0, 0), (1, 0), (0, 256 * 1024)])
def test_heff_apply_merged_and_separate_intermediates(device, merge_off, budget):
    """First-round intermediates merged into wide matrices (stacked right operands
    copied at prepare) or kept one per middle operator: sigma and diag equal the
    oracle either way, also with chunked intermediates."""
    print(f"[heff_apply merge_off={merge_off} budget={budget}]", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob = _problem(5, True)
    res = _run_heff(device, *prob, budget=budget, diag=True, merge_off=merge_off, variant=1, kseg=64)
    _close(res["sigma"], _dense_sigma(*prob))
    d = contract.heff_diag(contract.dense_env(L, lb), contract.dense_mpo(W1, len(Ldq), len(Mdq)),
                           contract.dense_mpo(W2, len(Mdq), len(Rdq)), contract.dense_env(R, rb))
    _close(res["diag"], mps.two_site_blocks_from_dense(d, lb, rb, two_site_blocks(lb, rb)))


def test_released_workspace_is_allocated_and_prepared_again(device):
    """A cached plan whose workspace was released gives the same sigma after
    ensure_workspace() and prepare(); before prepare it is refused."""
    import torch
    from paper_2310_03920_amd import _lib as X
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(5, True)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2).upload(device)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    s1, s2 = torch.empty_like(pt), torch.empty_like(pt)
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pt, s1)
    plan.release_workspace()
    with pytest.raises(RuntimeError, match="upload"):
        plan.apply(Lt, Rt, pt, s2)
    plan.ensure_workspace()
    with pytest.raises(RuntimeError, match="prepare"):
        plan.apply(Lt, Rt, pt, s2)
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pt, s2)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)


@pytest.mark.parametrize("roots,variant", [(3, 0), (2, 1)])
def test_heff_apply_multi_root(device, roots, variant):
    """R vectors per call (roots side by side in every column block): each root's
    sigma equals the oracle's."""
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[heff_apply multi-root] R={roots} variant={variant}", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(1, True)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, kernel_variant=variant, n_roots=roots).upload(device)
    rng = np.random.default_rng(31)
    psis = [psi] + [random_psi(lb, rb, rng) for _ in range(roots - 1)]
    pm = torch.from_numpy(X.pack_roots(lbB, rbB, [X.pack_psi(lbB, rbB, q) for q in psis])).to(device)
    assert pm.numel() == plan.info.psi_nnz
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    sm = torch.full_like(pm, float("nan"))
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pm, sm)
    torch.cuda.synchronize()
    for q, flat in zip(psis, X.unpack_roots(lbB, rbB, sm.cpu().numpy(), roots)):
        _close(X.unpack_psi(lbB, rbB, flat), _dense_sigma(lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, q))


def test_heff_diag_random_operands(device):
    print("[heff_diag]", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(4, True)
    got = _run_heff(device, lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi, diag=True)["diag"]
    d = contract.heff_diag(contract.dense_env(L, lb), contract.dense_mpo(W1, len(Ldq), len(Mdq)),
                           contract.dense_mpo(W2, len(Mdq), len(Rdq)), contract.dense_env(R, rb))
    _close(got, mps.two_site_blocks_from_dense(d, lb, rb, two_site_blocks(lb, rb)))


def test_heff_apply_is_bitwise_repeatable(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    print("[heff repeat]", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(5, True)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2).upload(device)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    plan.prepare(Lt, Rt)
    s1, s2 = torch.empty_like(pt), torch.empty_like(pt)
    plan.apply(Lt, Rt, pt, s1)
    plan.apply(Lt, Rt, pt, s2)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)


@pytest.mark.parametrize("direction", [0, 1])
def test_env_update_random_operands(device, direction):
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[env_update] direction={direction}", flush=True)
    rng = np.random.default_rng(10 + direction)
    kb = sorted([((2, 0), 64), ((2, 2), 3), ((3, 1), 70), ((3, -1), 1), ((4, 0), 9)])
    kb1 = sorted([((3, 1), 65), ((3, -1), 2), ((4, 0), 130), ((4, 2), 5), ((5, 1), 7), ((5, -1), 1)])
    din = [DQS[i % 9] for i in range(6)]
    dout = [DQS[(i * 4 + 1) % 9] for i in range(8)]
    if direction == 0:
        env = random_env(kb, din, rng)
        W = random_site_ops(din, dout, rng, per_col=3)
        A = random_site_tensor(kb, kb1, rng)
        ref = contract.env_blocks_from_dense(
            contract.env_update_left(contract.dense_env(env, kb), contract.dense_mpo(W, len(din), len(dout)),
                                     mps.dense_site_tensor(A, kb, kb1)), kb1, dout)
        bin_, bout = X.Bond(kb), X.Bond(kb1)
        plan = X.EnvPlan(0, bin_, bout, din, dout, W).upload(device)
        site = torch.from_numpy(X.pack_site(bin_, bout, A)).to(device)
    else:
        env = random_env(kb1, din, rng)
        W = random_site_ops(dout, din, rng, per_col=3)  # rows: ops at cut k, cols: ops at cut k+1
        B = random_site_tensor(kb, kb1, rng)
        ref = contract.env_blocks_from_dense(
            contract.env_update_right(contract.dense_env(env, kb1), contract.dense_mpo(W, len(dout), len(din)),
                                      mps.dense_site_tensor(B, kb, kb1)), kb, dout)
        bin_, bout = X.Bond(kb1), X.Bond(kb)
        plan = X.EnvPlan(1, bin_, bout, din, dout, W).upload(device)
        site = torch.from_numpy(X.pack_site(bout, bin_, B)).to(device)
    et = torch.from_numpy(X.pack_env(bin_, din, env)).to(device)
    out = torch.full((int(plan.info.out_nnz),), float("nan"), dtype=torch.float64, device=device)
    plan.update(et, site, out)
    got = X.unpack_env(bout, dout, out.cpu().numpy())
    scale = max(np.abs(blk).max() for op in ref for blk in op["blocks"].values())
    for a, op in enumerate(ref):
        for isrc, blk in op["blocks"].items():
            assert np.abs(got[a]["blocks"][isrc] - blk).max() <= RTOL * scale, (a, isrc)


def test_dots_match_numpy(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    print("[dots]", flush=True)
    rng = np.random.default_rng(0)
    for n in (1, 255, 70001):
        a = rng.standard_normal((5, n))
        b = rng.standard_normal(n)
        ws = torch.empty(X.davidson_ws_bytes(n, 32) // 8, dtype=torch.float64, device=device)
        out = torch.empty(5, dtype=torch.float64, device=device)
        X.dots(torch.from_numpy(a).to(device), torch.from_numpy(b).to(device), ws, out)
        ref = a @ b
        np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-13, atol=1e-13 * np.abs(a).sum())


@pytest.mark.parametrize("tail", ["kept", "garbage", "rotated"])
def test_davidson_step_matches_oracle(device, tail):
    """Steps k = 1 .. 8 on a growing basis equal the oracle's Davidson step.  The
    eigensolve of step k starts from step k-1's eigenvectors kept in the workspace
    tail; with that tail overwritten by non-orthonormal values (ignored) or by an
    unrelated orthogonal matrix (a valid start) the results are the same."""
    import torch
    from paper_2310_03920_amd import _lib as X
    print(f"[davidson_step] tail {tail}", flush=True)
    rng = np.random.default_rng(3)
    n, kmax = 3001, 8
    H = np.diag(np.linspace(-3, 5, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, 6)))
    H += 0.05 * (Q @ np.diag(rng.standard_normal(6)) @ Q.T)
    d = np.diag(H).copy()
    V = np.zeros((kmax, n))
    S = np.zeros((kmax, n))
    ws = torch.zeros(X.davidson_ws_bytes(n, kmax) // 8, dtype=torch.float64, device=device)
    dt = torch.from_numpy(d).to(device)
    x = torch.empty(n, dtype=torch.float64, device=device)
    hx, t = torch.empty_like(x), torch.empty_like(x)
    scal = torch.zeros(4, dtype=torch.float64, device=device)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    V[0], S[0] = v, H @ v
    Vt = torch.from_numpy(V).to(device)
    St = torch.from_numpy(S).to(device)
    qn = 32 * 32 + 1  # eigenvector tail of the workspace: 32 x 32 row-major, then k
    for k in range(1, kmax + 1):
        if k >= 3 and tail != "kept":
            q = np.zeros((32, 32))
            if tail == "garbage":
                q[:k - 1, :k - 1] = rng.standard_normal((k - 1, k - 1))
            else:
                q[:k - 1, :k - 1] = np.linalg.qr(rng.standard_normal((k - 1, k - 1)))[0]
            ws[-qn:] = torch.from_numpy(np.append(q.ravel(), k - 1.0)).to(device)
        X.davidson_step(n, k, kmax, Vt, St, dt, 1e-8, ws, x, hx, t, scal)
        theta, rn, xr, hxr, tr, tn = davidson.step(V[:k], S[:k], d, 1e-8)
        sc = scal.cpu().numpy()
        assert abs(sc[0] - theta) <= 1e-12 * max(1.0, abs(theta))
        assert abs(sc[1] - rn) <= 1e-10 * max(1.0, rn)
        np.testing.assert_allclose(x.cpu().numpy(), xr, atol=1e-10)
        np.testing.assert_allclose(hx.cpu().numpy(), hxr, atol=1e-10)
        np.testing.assert_allclose(t.cpu().numpy(), tr, atol=1e-9)
        if k < kmax:
            tv = t.cpu().numpy()
            V[k], S[k] = tv, H @ tv
            Vt[k] = torch.from_numpy(V[k]).to(device)
            St[k] = torch.from_numpy(S[k]).to(device)


@pytest.mark.parametrize("i,switch", [(1, None), (3, None), (5, None), (2, 4), (3, 4), (5, 4)])
def test_sigma_with_gpu_environments_equals_PtHP(device, i, switch):
    """Product MPO + GPU environment chain + GPU sigma == P^T H P psi (definition),
    for the NC MPO and for the NC->CN switch at cut 4 (Sec. II.B.2): sites (2, 3)
    have NC operators on all three cuts, (3, 4) the switch cut on the right, (5, 6)
    CN operators on all three."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.engine import Engine, site_payload
    from paper_2310_03920_amd.mpo import build_mpo
    print(f"[sigma vs PtHP] i={i} switch={switch}", flush=True)
    K, Mb = 8, 64
    h, g = make_integrals(K, seed=0)
    bonds = bond_sector_tables(K, K, 0, Mb)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    eng = Engine(build_mpo(h, g, switch=switch), device=device)
    eng.init_boundaries()
    for k in range(i):
        eng.update_left(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], left[k], device))
    for k in range(K - 1, i + 1, -1):
        eng.update_right(k, bonds[k], bonds[k + 1], site_payload(bonds[k], bonds[k + 1], right[k], device))
    plan = eng.heff_plan(i, bonds[i], bonds[i + 2])
    rng = np.random.default_rng(7)
    psi = random_psi(bonds[i], bonds[i + 2], rng)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    pt = torch.from_numpy(X.pack_psi(lb, rb, psi)).to(device)
    st = torch.empty_like(pt)
    plan.prepare(eng.left[i], eng.right[i + 2])
    plan.apply(eng.left[i], eng.right[i + 2], pt, st)
    got = X.unpack_psi(lb, rb, st.cpu().numpy())
    emb = mps.Embedding(h, g, K, 0, left[:i], right[i + 2:], bonds, i)
    keys = two_site_blocks(bonds[i], bonds[i + 2])
    ref = mps.two_site_blocks_from_dense(emb.apply(mps.dense_two_site(psi, bonds[i], bonds[i + 2])),
                                         bonds[i], bonds[i + 2], keys)
    _close(got, ref)
    # Hermiticity of the GPU H_eff: <phi|H psi> = <H phi|psi>
    phi = random_psi(bonds[i], bonds[i + 2], rng)
    ft = torch.from_numpy(X.pack_psi(lb, rb, phi)).to(device)
    hf = torch.empty_like(ft)
    plan.apply(eng.left[i], eng.right[i + 2], ft, hf)
    a = float(torch.dot(ft, st))
    b = float(torch.dot(hf, pt))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b) + 1)


@pytest.mark.parametrize("nparts", [3, 4])
def test_middle_bond_parts_sum_to_sigma_and_match_the_oracle(device, nparts):
    """Plans restricted to the middle-bond operators b = p (mod nparts): each part's
    sigma and diag equal the block-sparse oracle's sum over the same b, and the parts
    add up to the whole (the per-GPU share of a split over normal and complementary
    operators, with one sum of sigma)."""
    import torch
    from oracle import blocks
    from paper_2310_03920_amd import _lib as X
    print(f"[b parts] {nparts}", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob = _problem(4, True)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    total = torch.zeros_like(pt)
    dtotal = torch.zeros_like(pt)
    full = _dense_sigma(*prob)
    for p in range(nparts):
        plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, kernel_variant=1, split_kseg_min=16,
                          b_part=p, b_nparts=nparts).upload(device)
        st = torch.full_like(pt, float("nan"))
        dt = torch.full_like(pt, float("nan"))
        plan.prepare(Lt, Rt)
        plan.apply(Lt, Rt, pt, st)
        plan.diag(Lt, Rt, dt)
        torch.cuda.synchronize()
        got = X.unpack_psi(lbB, rbB, st.cpu().numpy())
        ref = blocks.heff_apply(lb, rb, L, W1, W2, R, psi, bsel=range(p, len(Mdq), nparts))
        ref = {k: ref.get(k, np.zeros_like(v)) for k, v in full.items()}
        scale = max(float(np.abs(v).max()) for v in full.values())
        for k in full:
            assert np.abs(got[k] - ref[k]).max() <= RTOL * scale, (p, k)
        total += st
        dtotal += dt
    _close(X.unpack_psi(lbB, rbB, total.cpu().numpy()), full)
    d = contract.heff_diag(contract.dense_env(L, lb), contract.dense_mpo(W1, len(Ldq), len(Mdq)),
                           contract.dense_mpo(W2, len(Mdq), len(Rdq)), contract.dense_env(R, rb))
    _close(X.unpack_psi(lbB, rbB, dtotal.cpu().numpy()), mps.two_site_blocks_from_dense(d, lb, rb, two_site_blocks(lb, rb)))


def test_binding_refuses_apply_before_prepare(device):
    """The mixed operators that sigma, diag and the adjoint read are written by
    prepare(L, R); an uploaded plan that was never prepared is refused on the host."""
    import torch
    from paper_2310_03920_amd import _lib as X
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(2)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    st = torch.empty_like(pt)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2).upload(device)
    for call in (lambda: plan.apply(Lt, Rt, pt, st), lambda: plan.diag(Lt, Rt, st),
                 lambda: plan.lower_f32(Lt, Rt)):
        with pytest.raises(RuntimeError, match="prepare"):
            call()
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, pt, st)
    plan.upload(device)  # a fresh workspace holds no mixed operators
    with pytest.raises(RuntimeError, match="prepare"):
        plan.apply(Lt, Rt, pt, st)
    torch.cuda.synchronize()
