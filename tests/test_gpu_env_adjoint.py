"""The adjoint of the environment update on the GPU (the chain of gradients through
environments, Sec. II.E.1).

For a cotangent G of the updated environment, f = <G, env_update(A, E, W)> is
linear in the input environment E and in the MPO values W and quadratic in the
site tensor A, so its directional derivatives are exact differences of the
oracle's environment update: f(E + V) - f(E), f(W + V) - f(W) and
(f(A + V) - f(A - V)) / 2.  Engine.env_update_backward (one-site sigma and its
adjoint with G as the opposite environment, plus layout moves and an axpy in
library kernels) must reproduce them for both directions.
"""

import numpy as np
import pytest

from oracle import contract, mps
from synth.blocks import random_env, random_site_ops, random_site_tensor

from test_gpu_parity import DQS

pytestmark = pytest.mark.gpu


def _f(direction, env, W, A, G, kb, kb1, din, dout, wrows, wcols):
    """<G, env_update> from the oracle's dense environment update."""
    Wd = contract.dense_mpo(W, len(wrows), len(wcols))
    if direction == 0:
        out = contract.env_update_left(contract.dense_env(env, kb), Wd, mps.dense_site_tensor(A, kb, kb1))
        Gd = contract.dense_env(G, kb1)
    else:
        out = contract.env_update_right(contract.dense_env(env, kb1), Wd, mps.dense_site_tensor(A, kb, kb1))
        Gd = contract.dense_env(G, kb)
    return float(np.sum(Gd * out))


def _axpy_env(env, V, t):
    return [{"dq": op["dq"], "blocks": {k: b + t * V[a]["blocks"][k] for k, b in op["blocks"].items()}}
            for a, op in enumerate(env)]


@pytest.mark.parametrize("direction", [0, 1])
def test_env_update_adjoint_matches_oracle_differences(device, direction):
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.engine import Engine
    from paper_2310_03920_amd.mpo import MPO, SiteMPO
    print(f"[env adjoint] direction={direction}", flush=True)
    rng = np.random.default_rng(40 + direction)
    kb = sorted([((2, 0), 17), ((2, 2), 3), ((3, 1), 70), ((3, -1), 1), ((4, 0), 9)])
    kb1 = sorted([((3, 1), 65), ((3, -1), 2), ((4, 0), 33), ((4, 2), 5), ((5, 1), 7), ((5, -1), 1)])
    din = [DQS[i % 9] for i in range(6)]
    dout = [DQS[(i * 4 + 1) % 9] for i in range(8)]
    if direction == 0:      # left[k] on kb (ops din) -> left[k+1] on kb1 (ops dout)
        cut_k, cut_k1 = din, dout
        env = random_env(kb, din, rng)
        G = random_env(kb1, dout, rng)
        env_bond, g_bond = kb, kb1
    else:                   # right[k+1] on kb1 (ops din) -> right[k] on kb (ops dout)
        cut_k, cut_k1 = dout, din
        env = random_env(kb1, din, rng)
        G = random_env(kb, dout, rng)
        env_bond, g_bond = kb1, kb
    W = random_site_ops(cut_k, cut_k1, rng, per_col=3)
    A = random_site_tensor(kb, kb1, rng)
    mpo = MPO(K=1, cuts=[list(range(len(cut_k))), list(range(len(cut_k1)))],
              sites=[SiteMPO(np.array([w[0] for w in W]), np.array([w[1] for w in W]),
                             np.array([w[2] for w in W]))],
              dq=[np.array(cut_k), np.array(cut_k1)])
    eng = Engine(mpo, device=device)
    kbB, kb1B = X.Bond(kb), X.Bond(kb1)
    site = torch.from_numpy(X.pack_site(kbB, kb1B, A)).to(device)
    env_t = torch.from_numpy(X.pack_env(X.Bond(env_bond), din, env)).to(device)
    G_t = torch.from_numpy(X.pack_env(X.Bond(g_bond), dout, G)).to(device)
    d_env, d_site, d_w = eng.env_update_backward(direction, 0, kb, kb1, site, env_t, G_t)
    torch.cuda.synchronize()
    d_env, d_site, d_w = d_env.cpu().numpy(), d_site.cpu().numpy(), d_w.cpu().numpy()

    f = lambda e, w, a: _f(direction, e, w, a, G, kb, kb1, din, dout, cut_k, cut_k1)  # noqa: E731
    f0 = f(env, W, A)
    scale = abs(f0) + 1.0
    # input environment (linear)
    V = random_env(env_bond, din, rng)
    got = float(np.dot(d_env, X.pack_env(X.Bond(env_bond), din, V)))
    ref = f(_axpy_env(env, V, 1.0), W, A) - f0
    print(f"d env: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale
    # site tensor (quadratic: the central difference is exact)
    VA = random_site_tensor(kb, kb1, rng)
    got = float(np.dot(d_site, X.pack_site(kbB, kb1B, VA)))
    Ap = {k: A[k] + VA[k] for k in A}
    Am = {k: A[k] - VA[k] for k in A}
    ref = 0.5 * (f(env, W, Ap) - f(env, W, Am))
    print(f"d site: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale
    # MPO values (linear), perturbing only the nonzero values
    VW = [(a, b, np.where(op != 0.0, rng.standard_normal((4, 4)), 0.0)) for a, b, op in W]
    got = float(sum(np.sum(d_w[e] * VW[e][2]) for e in range(len(W))))
    ref = f(env, [(a, b, op + VW[e][2]) for e, (a, b, op) in enumerate(W)], A) - f0
    print(f"d W: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale


def test_autograd_chains_through_two_environment_updates(device):
    """f = <G, left[k+2]> with left[k+2] = upd(upd(left[k], A_k), A_k+1): autograd
    gradients with respect to A_k, left[k] and the first site's MPO values equal
    exact differences of the same chain built from the oracle's update."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.autograd import EnvUpdateOperator
    from paper_2310_03920_amd.engine import Engine
    from paper_2310_03920_amd.mpo import MPO, SiteMPO
    print("[env adjoint] autograd chain of two left updates", flush=True)
    rng = np.random.default_rng(77)
    b0 = sorted([((2, 0), 9), ((2, 2), 3), ((3, 1), 12), ((3, -1), 1)])
    b1 = sorted([((3, 1), 10), ((3, -1), 2), ((4, 0), 14), ((4, 2), 5), ((5, 1), 3)])
    b2 = sorted([((4, 0), 11), ((4, 2), 4), ((5, 1), 13), ((5, -1), 6), ((6, 0), 2)])
    d0 = [DQS[i % 9] for i in range(5)]
    d1 = [DQS[(i * 4 + 1) % 9] for i in range(7)]
    d2 = [DQS[(i * 2 + 3) % 9] for i in range(6)]
    W0 = random_site_ops(d0, d1, rng, per_col=3)
    W1 = random_site_ops(d1, d2, rng, per_col=3)
    site = lambda W: SiteMPO(np.array([w[0] for w in W]), np.array([w[1] for w in W]),  # noqa: E731
                             np.array([w[2] for w in W]))
    mpo = MPO(K=2, cuts=[list(range(len(d))) for d in (d0, d1, d2)], sites=[site(W0), site(W1)],
              dq=[np.array(d) for d in (d0, d1, d2)])
    E0 = random_env(b0, d0, rng)
    A0 = random_site_tensor(b0, b1, rng)
    A1 = random_site_tensor(b1, b2, rng)
    G = random_env(b2, d2, rng)
    eng = Engine(mpo, device=device)
    B0, B1, B2 = X.Bond(b0), X.Bond(b1), X.Bond(b2)
    u0 = EnvUpdateOperator(eng, 0, 0, b0, b1)
    u1 = EnvUpdateOperator(eng, 0, 1, b1, b2)
    e0 = torch.from_numpy(X.pack_env(B0, d0, E0)).to(device).requires_grad_(True)
    a0 = torch.from_numpy(X.pack_site(B0, B1, A0)).to(device).requires_grad_(True)
    a1 = torch.from_numpy(X.pack_site(B1, B2, A1)).to(device)
    w0 = u0.values().requires_grad_(True)
    g = torch.from_numpy(X.pack_env(B2, d2, G)).to(device)
    e2 = u1(u0(e0, a0, w0), a1, u1.values())
    torch.dot(g, e2).backward()
    torch.cuda.synchronize()

    def f(E, A, W):
        e1 = contract.env_update_left(contract.dense_env(E, b0), contract.dense_mpo(W, len(d0), len(d1)),
                                      mps.dense_site_tensor(A, b0, b1))
        e2d = contract.env_update_left(e1, contract.dense_mpo(W1, len(d1), len(d2)),
                                       mps.dense_site_tensor(A1, b1, b2))
        return float(np.sum(contract.dense_env(G, b2) * e2d))

    f0 = f(E0, A0, W0)
    scale = abs(f0) + 1.0
    VA = random_site_tensor(b0, b1, rng)
    got = float(np.dot(a0.grad.cpu().numpy(), X.pack_site(B0, B1, VA)))
    ref = 0.5 * (f(E0, {k: A0[k] + VA[k] for k in A0}, W0) - f(E0, {k: A0[k] - VA[k] for k in A0}, W0))
    print(f"d A_k: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale
    VE = random_env(b0, d0, rng)
    got = float(np.dot(e0.grad.cpu().numpy(), X.pack_env(B0, d0, VE)))
    ref = f(_axpy_env(E0, VE, 1.0), A0, W0) - f0
    print(f"d left[k]: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale
    VW = [(a, b, np.where(op != 0.0, rng.standard_normal((4, 4)), 0.0)) for a, b, op in W0]
    got = float(np.sum(w0.grad.cpu().numpy() * np.array([v[2] for v in VW])))
    ref = f(E0, A0, [(a, b, op + VW[e][2]) for e, (a, b, op) in enumerate(W0)]) - f0
    print(f"d W_k: {got:.12e} vs {ref:.12e}", flush=True)
    assert abs(got - ref) <= 1e-11 * scale
