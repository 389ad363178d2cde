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
