"""Device-side state of a two-site sweep: environments, plans and site tensors.

Thin orchestration over the HIP library: plans are built on the host once per
(site, bond tables) and cached; every contraction is a library call on the
current HIP stream.  Environments live in HBM as flat payloads in the library's
layout (include/heffx.h).
"""

import numpy as np

from . import _lib as X
from . import mpo as M


class Engine:
    """Environments of one MPO on the GPU.

    left[k]  : payload of the left environment at cut k (ops mpo.cuts[k], bond k)
    right[k] : payload of the right environment at cut k (ops mpo.cuts[k], bond k)
    """

    # plan options of the sigma-vector, adjoint and environment plans: the one-buffer
    # pipeline with 512-element split-K segments (what the autotuner picks for the
    # large middle-chain problems)
    PLAN_OPTS = {"kernel_variant": 1, "split_kseg_min": 512}

    def __init__(self, mpo, device="cuda", t_budget_bytes=0, plan_opts=None):
        import torch
        self.torch = torch
        self.mpo = mpo
        self.K = mpo.K
        self.device = device
        self.t_budget = t_budget_bytes
        self.opts = dict(self.PLAN_OPTS if plan_opts is None else plan_opts)
        self.left = {}
        self.right = {}
        self._env_plans = {}
        self._heff_plans = {}
        self._pending = {}   # heff plan key -> future of its host build
        # one cached plan per site and kind: bond tables change with every
        # truncation, so a plan for older tables of the same site is dropped when
        # the new one is made (device tables and workspace are freed with it)
        self._latest = {}
        self._pool = None
        self._w = [X.MpoSite(s.rows, s.cols, s.mats) for s in mpo.sites]

    # -- boundaries: the vacuum bond carries the identity, the full bond carries H
    def init_boundaries(self):
        t = self.torch
        self.left[0] = t.ones(1, dtype=t.float64, device=self.device)
        self.right[self.K] = t.ones(1, dtype=t.float64, device=self.device)

    @staticmethod
    def _bkey(bond):
        return tuple((tuple(q), int(m)) for q, m in bond)

    def _keep_latest(self, cache, slot, key):
        old = self._latest.get(slot)
        if old is not None and old != key:
            cache.pop(old, None)
        self._latest[slot] = key

    def _build_env(self, direction, k, bond_k, bond_k1):
        if direction == 0:
            return X.EnvPlan(0, bond_k, bond_k1, self.mpo.dq[k], self.mpo.dq[k + 1], self._w[k],
                             t_budget_bytes=self.t_budget, **self.opts)
        return X.EnvPlan(1, bond_k1, bond_k, self.mpo.dq[k + 1], self.mpo.dq[k], self._w[k],
                         t_budget_bytes=self.t_budget, **self.opts)

    def _submit(self, fn, *args):
        if self._pool is None:
            from concurrent.futures import ThreadPoolExecutor
            self._pool = ThreadPoolExecutor(max_workers=2, thread_name_prefix="heffx-plan")
        return self._pool.submit(fn, *args)

    def prefetch_env_plan(self, direction, k, bond_k, bond_k1):
        """Start the host build of an environment-update plan on a worker thread (as
        prefetch_heff_plan); env_plan collects it."""
        key = ("env", direction, k, self._bkey(bond_k), self._bkey(bond_k1))
        if (direction, k, self._bkey(bond_k), self._bkey(bond_k1)) in self._env_plans or key in self._pending:
            return
        self._pending[key] = self._submit(self._build_env, direction, k, list(bond_k), list(bond_k1))

    def env_plan(self, direction, k, bond_k, bond_k1):
        key = (direction, k, self._bkey(bond_k), self._bkey(bond_k1))
        p = self._env_plans.get(key)
        if p is None:
            self._keep_latest(self._env_plans, ("env", direction, k), key)
            fut = self._pending.pop(("env",) + key, None)
            p = (fut.result() if fut is not None else self._build_env(direction, k, bond_k, bond_k1)).upload(self.device)
            self._env_plans[key] = p
        return p

    def _build_heff(self, i, bond_i, bond_i2):
        return X.HeffPlan(bond_i, bond_i2, self.mpo.dq[i], self.mpo.dq[i + 1], self.mpo.dq[i + 2],
                          self._w[i], self._w[i + 1], t_budget_bytes=self.t_budget, **self.opts)

    def prefetch_heff_plan(self, i, bond_i, bond_i2):
        """Start the host build of the sigma-vector plan of sites (i, i+1) on a
        worker thread (the library's plan builder is host-only and reentrant, and
        the binding releases the GIL during the call), so that it overlaps the
        environment plan and update that come first; heff_plan collects it and
        uploads it on the calling thread."""
        key = (i, self._bkey(bond_i), self._bkey(bond_i2))
        if key in self._heff_plans or key in self._pending:
            return
        self._pending[key] = self._submit(self._build_heff, i, list(bond_i), list(bond_i2))

    def heff_plan(self, i, bond_i, bond_i2):
        key = (i, self._bkey(bond_i), self._bkey(bond_i2))
        p = self._heff_plans.get(key)
        if p is None:
            fut = self._pending.pop(key, None)
            p = fut.result() if fut is not None else self._build_heff(i, bond_i, bond_i2)
            self._keep_latest(self._heff_plans, ("heff", i), key)
            p.upload(self.device)
            self._heff_plans[key] = p
        return p.ensure_workspace()

    def heff1_plan(self, i, bond_i, bond_i1):
        """One-site sigma-vector plan at site i (left environment at cut i, right at cut i+1)."""
        key = ("one", i, self._bkey(bond_i), self._bkey(bond_i1))
        p = self._heff_plans.get(key)
        if p is None:
            self._keep_latest(self._heff_plans, ("one", i), key)
            p = X.Heff1Plan(bond_i, bond_i1, self.mpo.dq[i], self.mpo.dq[i + 1], self._w[i],
                            t_budget_bytes=self.t_budget, **self.opts).upload(self.device)
            self._heff_plans[key] = p
        return p.ensure_workspace()

    def vjp_plan(self, i, bond_i, bond_i2):
        """Adjoint plan of the sigma-vector at sites (i, i+1) (built per call)."""
        return X.HeffVjpPlan(bond_i, bond_i2, self.mpo.dq[i], self.mpo.dq[i + 1], self.mpo.dq[i + 2],
                             self._w[i], self._w[i + 1], t_budget_bytes=self.t_budget,
                             **self.opts).upload(self.device)

    def env_update_backward(self, direction, k, bond_k, bond_k1, site, env_in, G):
        """Adjoint of update_left (direction 0: left[k] -> left[k+1]) or update_right
        (direction 1: right[k+1] -> right[k]) at site k.  For the cotangent G of the
        updated environment, f = <G, env_out> equals <A, H1 A> for the one-site
        H_eff of site k whose right (direction 0) or left (direction 1) environment is
        G, so the one-site sigma and its adjoint (with psi = g = A) give
          d env_in (payload layout), d site (site payload layout) = H1 A + H1^T A,
          d W_k (nnz, 4, 4: the values of the site's MPO tensor).
        Environments and site tensors stay on the device; every step is a library call."""
        torch = self.torch
        f64 = dict(dtype=torch.float64, device=self.device)
        lb, rb = X.Bond(bond_k), X.Bond(bond_k1)
        L, R = (env_in, G) if direction == 0 else (G, env_in)
        vjp = X.Heff1VjpPlan(lb, rb, self.mpo.dq[k], self.mpo.dq[k + 1], self._w[k],
                             t_budget_bytes=self.t_budget, **self.opts).upload(self.device)
        fwd = self.heff1_plan(k, bond_k, bond_k1)
        idx = torch.from_numpy(X.site_to_psi1_index(lb, rb)).to(self.device)
        n = int(vjp.info.psi_nnz)
        a = torch.empty(n, **f64)
        X.gather_index(idx, site, a)
        g_a = torch.empty(n, **f64)
        g_L = torch.empty(max(L.numel(), 1), **f64)
        g_R = torch.empty(max(R.numel(), 1), **f64)
        g_w = torch.empty(max(16 * vjp.nnz1, 1), **f64)
        g_w2 = torch.empty(max(16 * vjp.nnz2, 1), **f64)
        vjp.prepare(L, R)
        vjp.backward(L, R, a, a, g_a, g_L, g_R, g_w, g_w2)
        sig = torch.empty(n, **f64)
        fwd.prepare(L, R)
        fwd.apply(L, R, a, sig)
        X.axpy(1.0, sig, g_a)
        d_site = torch.zeros_like(site)
        X.scatter_index(idx, g_a, d_site)
        d_env = (g_L[:L.numel()] if direction == 0 else g_R[:R.numel()])
        return d_env, d_site, g_w[:16 * vjp.nnz1].view(vjp.nnz1, 4, 4)

    def drop_plans(self):
        for fut in self._pending.values():
            fut.result()
        self._pending.clear()
        self._env_plans.clear()
        self._heff_plans.clear()
        self._latest.clear()

    def update_left(self, k, bond_k, bond_k1, A):
        """left[k+1] from left[k] and the left-canonical tensor A (payload) of site k."""
        p = self.env_plan(0, k, bond_k, bond_k1)
        out = self.torch.empty(int(p.info.out_nnz), dtype=self.torch.float64, device=self.device)
        p.update(self.left[k], A, out)
        self.left[k + 1] = out
        return out

    def update_right(self, k, bond_k, bond_k1, B):
        """right[k] from right[k+1] and the right-canonical tensor B (payload) of site k."""
        p = self.env_plan(1, k, bond_k, bond_k1)
        out = self.torch.empty(int(p.info.out_nnz), dtype=self.torch.float64, device=self.device)
        p.update(self.right[k + 1], B, out)
        self.right[k] = out
        return out


def site_payload(bond_l, bond_r, tensor, device="cuda"):
    import torch
    return torch.from_numpy(X.pack_site(X.Bond(bond_l), X.Bond(bond_r), tensor)).to(device)


def mpo_from_integrals(h, g):
    return M.build_nc_mpo(np.asarray(h), np.asarray(g))
