"""hx_heff_apply_noalloc (prepare + apply with the library's static device scratch)
against hx_heff_prepare + hx_heff_apply with a caller workspace: bit for bit (same
kernels, same summation order), on calls in a row whose second problem is smaller
than the first, and again on the first after the smaller one has used the scratch."""

import numpy as np
import pytest

from synth import bond_sector_tables, make_integrals
from synth.blocks import random_env, random_psi

pytestmark = pytest.mark.gpu


def _case(K, M, i, seed, device):
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.engine import Engine
    from paper_2310_03920_amd.mpo import build_nc_mpo
    m = build_nc_mpo(*make_integrals(K, seed=seed))
    b = bond_sector_tables(K, K, 0, M)
    lb, rb = X.Bond(b[i]), X.Bond(b[i + 2])
    W1 = X.MpoSite(m.sites[i].rows, m.sites[i].cols, m.sites[i].mats)
    W2 = X.MpoSite(m.sites[i + 1].rows, m.sites[i + 1].cols, m.sites[i + 1].mats)
    plan = X.HeffPlan(lb, rb, m.dq[i], m.dq[i + 1], m.dq[i + 2], W1, W2, **Engine.PLAN_OPTS).upload(device)
    rng = np.random.default_rng(seed + 10)
    Ldq, Rdq = [tuple(x) for x in m.dq[i]], [tuple(x) for x in m.dq[i + 2]]
    L = torch.from_numpy(X.pack_env(lb, Ldq, random_env(b[i], Ldq, rng))).to(device)
    R = torch.from_numpy(X.pack_env(rb, Rdq, random_env(b[i + 2], Rdq, rng))).to(device)
    psi = torch.from_numpy(X.pack_psi(lb, rb, random_psi(b[i], b[i + 2], rng))).to(device)
    return plan, L, R, psi


def test_noalloc_sigma_equals_the_workspace_path(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    big = _case(6, 32, 2, 1, device)
    small = _case(4, 8, 1, 2, device)
    limit = 64 << 20
    assert small[0].info.ws_bytes < big[0].info.ws_bytes <= limit
    assert small[0].info.psi_nnz < big[0].info.psi_nnz
    for name, (plan, L, R, psi) in (("big", big), ("small", small), ("big again", big)):
        print(f"[noalloc] {name}: psi {plan.info.psi_nnz}, ws {plan.info.ws_bytes} bytes", flush=True)
        ref = torch.empty_like(psi)
        plan.prepare(L, R)
        plan.apply(L, R, psi, ref)
        got = torch.full_like(psi, float("nan"))
        plan.apply_noalloc(L, R, psi, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), float((got - ref).abs().max())
        assert float(ref.abs().max()) > 0
    X.lib()
