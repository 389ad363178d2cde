"""torch.autograd binding of the sigma-vector and its adjoint.

`HeffOperator` owns a forward plan and an adjoint (VJP) plan for one two-site
problem; calling it returns sigma = H_eff(L, W1, W2, R) psi as a tensor that
autograd differentiates through the library's hx_heff_apply_backward: the
gradients of any scalar built from sigma flow to psi, L, R and to the nonzero
MPO values W1 / W2 (Sec. II.C.1 operators; the energy gradient
d<psi|H_eff|psi> that reduced density matrices and orbital gradients need,
Sec. II.E.1).  The MPO values are compiled into the plans: the w1 / w2 tensors
passed in must hold the values the operator was built with (they exist to
receive gradients).  All arithmetic runs in the HIP library.
"""

import numpy as np
import torch

from . import _lib as X


class HeffOperator:
    def __init__(self, lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, device="cuda", **plan_opts):
        self.w1_site = W1 if isinstance(W1, X.MpoSite) else X.MpoSite.from_entries(W1)
        self.w2_site = W2 if isinstance(W2, X.MpoSite) else X.MpoSite.from_entries(W2)
        self.fwd = X.HeffPlan(lbond, rbond, Ldq, mid_dq, Rdq, self.w1_site, self.w2_site, **plan_opts).upload(device)
        self.vjp = X.HeffVjpPlan(lbond, rbond, Ldq, mid_dq, Rdq, self.w1_site, self.w2_site,
                                 **plan_opts).upload(device)
        self.device = device

    def values(self):
        """The MPO values the plans were built with, as device tensors (nnz, 4, 4)."""
        return (torch.from_numpy(self.w1_site.vals.reshape(-1, 4, 4).copy()).to(self.device),
                torch.from_numpy(self.w2_site.vals.reshape(-1, 4, 4).copy()).to(self.device))

    def __call__(self, L, R, w1, w2, psi):
        dev = self.fwd.device
        X.need(w1, "w1", 16 * self.vjp.nnz1, "float64", dev)
        X.need(w2, "w2", 16 * self.vjp.nnz2, "float64", dev)
        return _HeffApply.apply(self, L, R, w1, w2, psi)


class _HeffApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, L, R, w1, w2, psi):
        L, R, psi = L.contiguous(), R.contiguous(), psi.contiguous()
        sigma = torch.empty_like(psi)
        op.fwd.prepare(L, R)
        op.fwd.apply(L, R, psi, sigma)
        ctx.op = op
        ctx.w_shapes = (w1.shape, w2.shape)
        ctx.save_for_backward(L, R, psi)
        return sigma

    @staticmethod
    def backward(ctx, g):
        L, R, psi = ctx.saved_tensors
        op = ctx.op
        g = g.contiguous()
        g_psi = torch.empty_like(psi)
        g_L = torch.empty_like(L)
        g_R = torch.empty_like(R)
        g_w1 = torch.empty(max(16 * op.vjp.nnz1, 1), dtype=torch.float64, device=psi.device)
        g_w2 = torch.empty(max(16 * op.vjp.nnz2, 1), dtype=torch.float64, device=psi.device)
        op.vjp.prepare(L, R)
        op.vjp.backward(L, R, psi, g, g_psi, g_L, g_R, g_w1, g_w2)
        s1, s2 = ctx.w_shapes
        return (None, g_L, g_R, g_w1[:16 * op.vjp.nnz1].view(s1), g_w2[:16 * op.vjp.nnz2].view(s2), g_psi)


class EnvUpdateOperator:
    """The environment update of one site as an autograd operation.

    direction 0: left[k] (bond k) -> left[k+1] (bond k+1); direction 1: right[k+1]
    (bond k+1) -> right[k] (bond k).  Forward is hx_env_update; backward recomputes
    through the one-site sigma-vector and its adjoint (Engine.env_update_backward),
    so gradients chain through any number of environment updates to the site
    tensors, the first environment and the MPO values of every site.  The MPO values
    are compiled into the plans; the w tensor passed in (`values()`) receives
    gradients."""

    def __init__(self, engine, direction, k, bond_k, bond_k1):
        self.eng, self.direction, self.k = engine, direction, k
        self.bond_k, self.bond_k1 = bond_k, bond_k1
        self.plan = engine.env_plan(direction, k, bond_k, bond_k1)
        self.out_nnz = int(self.plan.info.out_nnz)

    def values(self):
        s = self.eng.mpo.sites[self.k]
        return torch.from_numpy(np.asarray(s.mats, dtype=np.float64).reshape(-1, 4, 4).copy()).to(self.eng.device)

    def __call__(self, env_in, site, w):
        X.need(w, "w", 16 * len(self.eng.mpo.sites[self.k].rows), "float64", self.plan.device)
        return _EnvUpdate.apply(self, env_in, site, w)


class _EnvUpdate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, env_in, site, w):
        env_in, site = env_in.contiguous(), site.contiguous()
        out = torch.empty(op.out_nnz, dtype=torch.float64, device=env_in.device)
        op.plan.update(env_in, site, out)
        ctx.op = op
        ctx.w_shape = w.shape
        ctx.save_for_backward(env_in, site)
        return out

    @staticmethod
    def backward(ctx, g):
        env_in, site = ctx.saved_tensors
        op = ctx.op
        d_env, d_site, d_w = op.eng.env_update_backward(op.direction, op.k, op.bond_k, op.bond_k1, site, env_in,
                                                        g.contiguous())
        return None, d_env, d_site, d_w.reshape(ctx.w_shape)
