"""The Python binding refuses malformed operands before a pointer reaches the
library (whose entry points take bare pointers with plan-implied lengths).  All
checks run on the host: the plans here are built but never uploaded, and no
device work is issued."""

import numpy as np
import pytest
import torch

from paper_2310_03920_amd import _lib as X
from paper_2310_03920_amd import mpo as M
from synth import bond_sector_tables, make_integrals


@pytest.fixture(scope="module")
def plans():
    K, i = 4, 1
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 16)
    heff = X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                      M.site_entries(m, i + 1))
    vjp = X.HeffVjpPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                        M.site_entries(m, i + 1))
    env = X.EnvPlan(0, b[i], b[i + 1], m.dq[i], m.dq[i + 1], M.site_entries(m, i))
    return heff, vjp, env


def _f64(n):
    return torch.zeros(max(int(n), 1), dtype=torch.float64)


def test_need_checks_type_dtype_layout_length_and_device():
    X.need(None, "x", 0)
    with pytest.raises(ValueError, match="missing"):
        X.need(None, "x", 3)
    with pytest.raises(TypeError):
        X.need(np.zeros(3), "x", 3)
    with pytest.raises(ValueError, match="dtype"):
        X.need(torch.zeros(3, dtype=torch.float32), "x", 3)
    with pytest.raises(ValueError, match="contiguous"):
        X.need(torch.zeros((3, 2), dtype=torch.float64).t(), "x", 3)
    with pytest.raises(ValueError, match="elements"):
        X.need(torch.zeros(2, dtype=torch.float64), "x", 3)
    with pytest.raises(ValueError, match="device"):
        X.need(torch.zeros(3, dtype=torch.float64), "x", 3)


def test_sigma_entry_points_refuse_bad_operands(plans):
    heff, _, _ = plans
    info = heff.info
    L, R = _f64(info.in_nnz), _f64(info.in2_nnz)
    psi, sig = _f64(info.psi_nnz), _f64(info.psi_nnz)
    with pytest.raises(ValueError, match="L: dtype"):
        heff.apply(L.float(), R, psi, sig)
    with pytest.raises(ValueError, match="R: .* elements"):
        heff.apply(L, R[:-1], psi, sig)
    with pytest.raises(ValueError, match="psi: .* elements"):
        heff.apply(L, R, psi[:-1], sig)
    with pytest.raises(ValueError, match="sigma: dtype"):
        heff.apply(L, R, psi, sig.float())
    with pytest.raises(ValueError, match="device"):
        heff.apply(L, R, psi, sig)          # host tensors
    with pytest.raises(ValueError, match="diag: .* elements"):
        heff.diag(L, R, psi[:-1])
    with pytest.raises(ValueError, match="psi: dtype"):
        heff.apply_f32(psi, sig.float())     # FP64 psi on the FP32 path
    with pytest.raises(ValueError, match="L: dtype"):
        heff.prepare(L.float(), R)


def test_adjoint_and_environment_entry_points_refuse_bad_operands(plans):
    _, vjp, env = plans
    info = vjp.info
    L, R = _f64(info.in_nnz), _f64(info.in2_nnz)
    psi, g, gp = _f64(info.psi_nnz), _f64(info.psi_nnz), _f64(info.psi_nnz)
    gL, gR = _f64(info.in_nnz), _f64(info.in2_nnz)
    gw1, gw2 = _f64(16 * vjp.nnz1), _f64(16 * vjp.nnz2)
    with pytest.raises(ValueError, match="g_W1: .* elements"):
        vjp.backward(L, R, psi, g, gp, gL, gR, gw1[:-1], gw2)
    with pytest.raises(ValueError, match="g_L: dtype"):
        vjp.backward(L, R, psi, g, gp, gL.float(), gR, gw1, gw2)
    with pytest.raises(ValueError, match="g: .* elements"):
        vjp.backward(L, R, psi, g[:-1], gp, gL, gR, gw1, gw2)
    ei = env.info
    with pytest.raises(ValueError, match="site: .* elements"):
        env.update(_f64(ei.in_nnz), _f64(ei.in2_nnz)[:-1], _f64(ei.out_nnz))
    with pytest.raises(ValueError, match="env_out: dtype"):
        env.update(_f64(ei.in_nnz), _f64(ei.in2_nnz), _f64(ei.out_nnz).float())


def test_davidson_step_refuses_bad_shapes():
    n, kmax = 10, 4
    V, S = torch.zeros((kmax, n), dtype=torch.float64), torch.zeros((kmax, n), dtype=torch.float64)
    v = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="kmax"):
        X.davidson_step(n, 5, kmax, V, S, v, 1e-8, v, v, v, v, v)
    with pytest.raises(ValueError, match="row-major"):
        X.davidson_step(n, 2, kmax, V[:, :5], S, v, 1e-8, v, v, v, v, v)
    with pytest.raises(ValueError, match="diag: .* elements"):
        X.davidson_step(n, 2, kmax, V, S, v[:3], 1e-8, v, v, v, v, v)


def test_noalloc_entry_point_rejects_a_workspace_above_its_static_scratch():
    """The no-allocation sigma-vector refuses plans whose workspace exceeds the
    library's static scratch (64 MiB) before touching the device."""
    K, i = 16, 7
    m = M.build_nc_mpo(*make_integrals(K, seed=0))
    b = bond_sector_tables(K, K, 0, 256)
    p = X.HeffPlan(b[i], b[i + 2], m.dq[i], m.dq[i + 1], m.dq[i + 2], M.site_entries(m, i),
                   M.site_entries(m, i + 1))
    assert p.info.ws_bytes > 64 << 20
    rc = X.lib().hx_heff_apply_noalloc(p.h, None, None, None, None, None)
    assert rc == X.HX_EINVAL
    assert "exceeds the static scratch" in X.lib().hx_last_error().decode()
