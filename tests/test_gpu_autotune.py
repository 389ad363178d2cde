"""The autotuner on the GPU: it returns options from its search space, and the
tuned plan's sigma equals the oracle's."""

import pytest

from test_gpu_parity import _close, _dense_sigma, _problem

pytestmark = pytest.mark.gpu


def test_tune_heff_returns_a_correct_plan(device):
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd import autotune as A
    print("[autotune] seed 1 big", flush=True)
    prob = _problem(1, True)
    lb, rb, Ldq, Mdq, Rdq, L, R, W1, W2, psi = prob
    lbB, rbB = X.Bond(lb), X.Bond(rb)
    Lt = torch.from_numpy(X.pack_env(lbB, Ldq, L)).to(device)
    Rt = torch.from_numpy(X.pack_env(rbB, Rdq, R)).to(device)
    pt = torch.from_numpy(X.pack_psi(lbB, rbB, psi)).to(device)
    best, timings = A.tune_heff(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, Lt, Rt, pt, reps=1)
    for name, values in A.AXES:
        assert best[name] in values
    assert len(timings) == 1 + sum(len(v) - 1 for _, v in A.AXES) and all(t is not None for t in timings.values())
    plan = X.HeffPlan(lbB, rbB, Ldq, Mdq, Rdq, W1, W2, **best).upload(device)
    plan.prepare(Lt, Rt)
    st = torch.empty_like(pt)
    plan.apply(Lt, Rt, pt, st)
    _close(X.unpack_psi(lbB, rbB, st.cpu().numpy()), _dense_sigma(*prob))
