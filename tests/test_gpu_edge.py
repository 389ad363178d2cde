"""Degenerate inputs of the sigma-vector path on the GPU.

* a two-site space with no allowed block (the target is out of reach of the
  bonds): the plan has psi_nnz = 0 and every call is a no-op that succeeds;
* an all-zero MPO site: sigma and diag are exactly zero -- every output tile is
  written (sigma is overwritten, never accumulated), also tiles with no task;
* the identity MPO: sigma reduces to the matrix products L psi R^T per block,
  checked against the oracle's dense contraction.
"""

import numpy as np
import pytest

from oracle import contract, mps
from synth.blocks import random_env, random_psi, two_site_blocks

from test_gpu_parity import _close, _dense_sigma, _problem, _run_heff

pytestmark = pytest.mark.gpu


def test_empty_two_site_space_is_a_noop(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    print("[edge] empty two-site space", flush=True)
    lb = [((0, 0), 3)]
    rb = [((9, 1), 2)]  # nine electrons more than the left block: out of reach of two sites
    rng = np.random.default_rng(0)
    _, _, Ldq, Mdq, Rdq, _, _, W1, W2, _ = _problem(0)
    assert not two_site_blocks(lb, rb)
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2).upload(device)
    assert plan.info.psi_nnz == 0 and plan.info.flops_apply == 0
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, random_env(lb, Ldq, rng))).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, random_env(rb, Rdq, rng))).to(device)
    e = torch.empty(0, dtype=torch.float64, device=device)
    plan.prepare(Lt, Rt)
    plan.apply(Lt, Rt, e, torch.empty_like(e))
    plan.diag(Lt, Rt, torch.empty_like(e))
    torch.cuda.synchronize()


def test_zero_mpo_gives_exact_zero_sigma_and_diag(device):
    print("[edge] all-zero MPO site", flush=True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = _problem(1, True)
    W1z = [(a, b, 0.0 * np.asarray(op)) for a, b, op in W1]
    res = _run_heff(device, lb, rb, Ldq, Mdq, Rdq, L, R, W1z, W2, psi, diag=True)
    for k in two_site_blocks(lb, rb):
        assert np.all(res["sigma"][k] == 0.0), k
        assert np.all(res["diag"][k] == 0.0), k


def test_identity_mpo_reduces_to_block_products(device):
    """W1 = W2 = identity on a single operator channel: sigma = (L_0 (x) 1) psi (R_0 (x) 1)^T."""
    print("[edge] identity MPO", flush=True)
    rng = np.random.default_rng(3)
    lb, rb = _problem(2, True)[:2]
    Ldq = Mdq = Rdq = [(0, 0)]
    L = random_env(lb, Ldq, rng)
    R = random_env(rb, Rdq, rng)
    eye = [(0, 0, np.eye(4))]
    psi = random_psi(lb, rb, rng)
    got = _run_heff(device, lb, rb, Ldq, Mdq, Rdq, L, R, eye, eye, psi)["sigma"]
    Ld, Rd = contract.dense_env(L, lb)[0], contract.dense_env(R, rb)[0]
    ref = np.einsum("xl,lstr,yr->xsty", Ld, mps.dense_two_site(psi, lb, rb), Rd)
    _close(got, mps.two_site_blocks_from_dense(ref, lb, rb, two_site_blocks(lb, rb)))
    _close(got, _dense_sigma(lb, rb, Ldq, Mdq, Rdq, L, R, eye, eye, psi))
