"""Two-site DMRG sweep driver (Sec. II.A.2) on top of the heffx library.

Per site step (sites i, i+1):
  plan   -- host: block tables and GEMM task lists (library, C++)
  prepare-- mixed complementary operators (GPU)
  diag   -- diag(H_eff) for the preconditioner (GPU)
  Davidson: sigma = H_eff psi (GPU) + Davidson step (GPU); only the three
            scalars theta, |r|, |t| are read back each iteration
  split  -- SVD of the two-site tensor per fused sector, keep the M largest
            singular values over all sectors (host LAPACK)
  env    -- environment update with the new canonical tensor (GPU)

Passes alternate: left-to-right i = i0..K-2, right-to-left i = K-3..0, where a
pass's end pair is split towards the next pass.
"""

import os
import threading
import time

import numpy as np

from . import _lib as X
from .engine import Engine, site_payload
from .mpo import SITE_QN, build_mpo


def _add(q, d, sign=1):
    return (q[0] + sign * d[0], q[1] + sign * d[1])


def contract_two(t1, t2, bl, bm, br):
    """Two adjacent one-site tensors -> two-site tensor {(il, s1, s2, ir): block}."""
    by_m = {}
    for (im, s2, ir), blk in t2.items():
        by_m.setdefault(im, []).append((s2, ir, blk))
    out = {}
    for (il, s1, im), a in t1.items():
        for s2, ir, b in by_m.get(im, []):
            key = (il, s1, s2, ir)
            v = a @ b
            out[key] = out[key] + v if key in out else v
    return out


def _fused_sectors(psi, bl, br):
    """Group two-site blocks by the label Q of the middle bond (left block + s1)."""
    groups = {}
    for (il, s1, s2, ir), blk in psi.items():
        Q = _add(bl[il][0], SITE_QN[s1])
        g = groups.setdefault(Q, {"rows": {}, "cols": {}, "blocks": []})
        g["rows"].setdefault((il, s1), bl[il][1])
        g["cols"].setdefault((s2, ir), br[ir][1])
        g["blocks"].append(((il, s1), (s2, ir), blk))
    for g in groups.values():
        g["rows"] = sorted(g["rows"].items())
        g["cols"] = sorted(g["cols"].items())
    return groups


def _matrix(g):
    ro, co = {}, {}
    o = 0
    for k, m in g["rows"]:
        ro[k] = o
        o += m
    nr = o
    o = 0
    for k, m in g["cols"]:
        co[k] = o
        o += m
    mat = np.zeros((nr, o))
    for rk, ck, blk in g["blocks"]:
        mat[ro[rk]:ro[rk] + blk.shape[0], co[ck]:co[ck] + blk.shape[1]] = blk
    return mat, ro, co


# Singular values closer than TIE_RTOL * (largest singular value) to the first
# value of a run of near-equal values are treated as equal.  A spin-free
# Hamiltonian gives exactly equal singular values for the members of a spin
# multiplet (different 2Sz sectors); rounding would otherwise decide which of them
# survive a cut through the multiplet.
TIE_RTOL = 1e-8


def _keep_order(cand):
    """cand: (-s, Q, j) sorted ascending.  Runs of values within TIE_RTOL * s_max of
    the run's first value are re-ordered by (sector, index)."""
    if not cand:
        return cand
    tol = TIE_RTOL * -cand[0][0]
    out, a = [], 0
    while a < len(cand):
        b = a + 1
        while b < len(cand) and cand[b][0] - cand[a][0] <= tol:
            b += 1
        out.extend(sorted(cand[a:b], key=lambda c: (c[1], c[2])))
        a = b
    return out


_svd_pool = None
_svd_lock = threading.Lock()


def _sector_svds(mats):
    """Full SVDs of the fused-sector matrices, several at once on a host thread pool
    with one BLAS thread each (LAPACK releases the GIL), largest first; the results
    do not depend on the scheduling."""
    global _svd_pool
    if len(mats) < 2:
        return [np.linalg.svd(m, full_matrices=True) for m in mats]
    from threadpoolctl import threadpool_limits
    with _svd_lock:
        if _svd_pool is None:
            from concurrent.futures import ThreadPoolExecutor
            _svd_pool = ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1)),
                                           thread_name_prefix="heffx-svd")
        order = sorted(range(len(mats)), key=lambda j: -mats[j].size)
        with threadpool_limits(limits=1, user_api="blas"):
            done = dict(zip(order, _svd_pool.map(lambda j: np.linalg.svd(mats[j], full_matrices=True), order)))
    return [done[j] for j in range(len(mats))]


def split(psi, bl, br, M, direction, fixed=None, info=None):
    """SVD split of a two-site tensor.

    direction 0: psi = A C with A left-canonical (new bond sectors from U);
    direction 1: psi = C B with B right-canonical (from V^T).
    Keeps the M largest singular values over all sectors, counting the zero
    singular values of the full (square) factor, ties (within TIE_RTOL) by
    (sector, index); with `fixed` = {Q: dim} the dims per sector are given instead.
    Returns (new_bond, canonical tensor, center tensor, discarded weight); with a
    dict `info`, info["kept_s"] receives the kept singular values (descending).
    """
    groups = _fused_sectors(psi, bl, br)
    cand = []
    fac = {}
    qs = sorted(groups)
    mats = [_matrix(groups[Q]) for Q in qs]
    svds = _sector_svds([m for m, _, _ in mats])
    for Q, (mat, ro, co), (U, S, Vt) in zip(qs, mats, svds):
        n = U.shape[0] if direction == 0 else Vt.shape[0]
        s_full = np.zeros(n)
        s_full[:len(S)] = S
        fac[Q] = (U, s_full, Vt, ro, co, groups[Q])
        for j in range(n):
            cand.append((-s_full[j], Q, j))
    if fixed is None:
        cand = _keep_order(sorted(cand))
        keep = cand[:M]
        kept = {}
        for _, Q, j in keep:
            kept[Q] = kept.get(Q, 0) + 1
        disc = float(sum(c[0] ** 2 for c in cand[M:]))
    else:
        kept = {Q: min(m, len(fac[Q][1])) for Q, m in fixed.items() if Q in fac}
        disc = float(sum((fac[Q][1][kept.get(Q, 0):] ** 2).sum() for Q in fac))
    new_bond = sorted((Q, m) for Q, m in kept.items() if m > 0)
    if info is not None:
        info["kept_s"] = sorted((float(x) for Q, m in new_bond for x in fac[Q][1][:m]), reverse=True)
    nidx = {Q: i for i, (Q, _) in enumerate(new_bond)}
    canon, center = {}, {}
    for Q, m in new_bond:
        U, s, Vt, ro, co, g = fac[Q]
        q = nidx[Q]
        if direction == 0:
            for (il, s1), mr in g["rows"]:
                canon[(il, s1, q)] = U[ro[(il, s1)]:ro[(il, s1)] + mr, :m].copy()
            Cm = s[:m, None] * np.vstack([Vt, np.zeros((max(0, m - Vt.shape[0]), Vt.shape[1]))])[:m]
            for (s2, ir), mc in g["cols"]:
                center[(q, s2, ir)] = Cm[:, co[(s2, ir)]:co[(s2, ir)] + mc].copy()
        else:
            for (s2, ir), mc in g["cols"]:
                canon[(q, s2, ir)] = Vt[:m, co[(s2, ir)]:co[(s2, ir)] + mc].copy()
            Ue = np.hstack([U, np.zeros((U.shape[0], max(0, m - U.shape[1])))])[:, :m]
            Cm = Ue * s[None, :m]
            for (il, s1), mr in g["rows"]:
                center[(il, s1, q)] = Cm[ro[(il, s1)]:ro[(il, s1)] + mr, :].copy()
    return new_bond, canon, center, disc


class Davidson:
    """GPU Davidson solver for one H_eff (all vector work in library kernels)."""

    def __init__(self, n, kmax=24, device="cuda"):
        import torch
        self.torch = torch
        self.n, self.kmax = n, kmax
        f64 = dict(dtype=torch.float64, device=device)
        self.V = torch.zeros((kmax, n), **f64)
        self.S = torch.zeros((kmax, n), **f64)
        # Ritz pairs of the current and the previous iteration (alternating buffers)
        self.xb = torch.zeros((2, n), **f64)
        self.hxb = torch.zeros((2, n), **f64)
        self.x, self.hx = self.xb[0], self.hxb[0]
        self.t = torch.zeros(n, **f64)
        self.scal = torch.zeros(4, **f64)
        self.ws = torch.zeros(max(X.davidson_ws_bytes(n, kmax) // 8, 1), **f64)
        # theta, |r|, |t| of a step, copied to pinned host memory behind an event
        self._scal_h = torch.zeros(3, dtype=torch.float64, pin_memory=True)
        self._scal_ev = torch.cuda.Event()

    def solve(self, matvec, psi0, diag, tol=1e-8, max_iter=30, guard=1e-8, on_iter=None, thick=True,
              queue_ahead=True):
        """Lowest eigenpair of the operator `matvec(v, out)`; returns (theta, rnorm, n_matvec).

        When the basis is full it restarts from the Ritz vector and, with `thick`,
        also the previous iteration's Ritz vector (orthogonalised against it; its
        H-image follows by linear combination, so the restart costs no
        sigma-vector; skipped when the two are nearly parallel, where that
        combination would lose precision).  With `queue_ahead`, steps far from
        convergence queue the next expansion before the host reads their scalars
        (same iterates).  The Ritz vector is left in self.x."""
        n, kmax = self.n, self.kmax
        V, S = self.V, self.S
        V[0].copy_(psi0)
        X.normalize(V[0], self.ws)
        matvec(V[0], S[0])
        nmv, k = 1, 1
        theta = rnorm = None
        cur = 0

        def step(kk, c):
            X.davidson_step(n, kk, kmax, V, S, diag, guard, self.ws, self.xb[c], self.hxb[c], self.t, self.scal)

        prev_r = None
        for it in range(max_iter):
            step(k, cur)
            # While the last residual is far above tol, the next expansion (the one
            # the loop issues next unless it stops here) is queued before the host
            # reads this step's scalars, so the GPU does not wait for the host's
            # decision; the iterates are unchanged, and that sigma-vector is wasted
            # only when this step ends the solve.
            ahead = (queue_ahead and k < kmax and it < max_iter - 1 and prev_r is not None
                     and prev_r > 100.0 * tol)
            if ahead:
                self._scal_h.copy_(self.scal[:3], non_blocking=True)
                self._scal_ev.record()
                V[k].copy_(self.t)
                matvec(V[k], S[k])
                self._scal_ev.synchronize()
                theta, rnorm, tnorm = self._scal_h.tolist()
            else:
                theta, rnorm, tnorm = (float(v) for v in self.scal[:3].cpu())
            prev_r = rnorm
            stop = bool(on_iter(it, theta, rnorm)) if on_iter else False
            if stop or rnorm < tol or it == max_iter - 1 or not (tnorm > 1e-14):
                break
            if k == kmax:
                prev = 1 - cur
                V[0].copy_(self.xb[cur])
                S[0].copy_(self.hxb[cur])
                k = 1
                if thick and it > 0:
                    X.davidson_restart2(self.xb[cur], self.hxb[cur], self.xb[prev], self.hxb[prev], V[1], S[1],
                                        self.ws, self.scal)
                    # the H-image of v1 is a difference of nearly parallel vectors when x has
                    # barely moved; use it only while its rounding stays far below tol
                    if float(self.scal[3].cpu()) > 1e-3:
                        step(1, prev)  # projected-matrix row 0 of the new basis
                        k = 2
                cur = 1 - cur
                step(k, cur)
            if not ahead:
                V[k].copy_(self.t)
                matvec(V[k], S[k])
            nmv += 1
            k += 1
            cur = 1 - cur
        self.x, self.hx = self.xb[cur], self.hxb[cur]
        return theta, rnorm, nmv

    def solve_mixed(self, mv32, mv64, psi0, diag, tol=1e-8, max_iter=30, low_tol=1e-5, guard=1e-8):
        """Reduced-precision sigma-vectors until |r| < low_tol or the phase stops
        paying, then FP64 sigma-vectors restarted from that Ritz vector until
        |r| < tol.  The phase stops paying when its last 6 iterations gained less
        than 2x in |r|: near the rounding floor of that precision, whose level
        grows with the operator's norm and size, or from a warm start already below
        it.  Returns (theta, rnorm, n_matvec_low, n_matvec_f64)."""
        hist = []

        def watch(it, theta, rn):
            hist.append(rn)
            return len(hist) >= 7 and rn > 0.5 * hist[-7]

        _, _, n32 = self.solve(mv32, psi0, diag, tol=low_tol, max_iter=max_iter, guard=guard,
                               on_iter=watch)
        x32 = self.x.clone()
        theta, rnorm, n64 = self.solve(mv64, x32, diag, tol=tol, max_iter=max_iter, guard=guard)
        return theta, rnorm, n32, n64


# Reduced-precision phase of the mixed Davidson per block-product precision:
# stop at |r| < low_tol, or on stagnation (6 iterations without a 2x gain).
PRECISIONS = {"f64": {}, "f32": {"low_tol": 1e-5}, "bf16": {"low_tol": 3e-3}}


class DMRG:
    """Two-site DMRG for H(h, g) in the (n_elec, twosz) sector at bond dimension M."""

    def __init__(self, h, g, n_elec, twosz, M, seed=0, device="cuda", tol=1e-8, max_iter=30, kmax=24,
                 bonds=None, tensors=None, t_budget_bytes=0, precision="f64", mpo_switch=None):
        from synth import bond_sector_tables, random_right_canonical_mps
        self.K = h.shape[0]
        self.M = M
        self.device = device
        self.tol, self.max_iter, self.kmax = tol, max_iter, kmax
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        self.h, self.g = np.asarray(h, dtype=np.float64), np.asarray(g, dtype=np.float64)
        # mpo_switch: None = NC partition at every cut; c = NC up to cut c and CN
        # after it (same operator, smaller bonds on the right half for c ~ K/2)
        self.mpo_switch = mpo_switch
        self.mpo = self._mpo(self.h, self.g)
        self.bonds = bonds if bonds is not None else bond_sector_tables(self.K, n_elec, twosz, M)
        self.tensors = tensors if tensors is not None else random_right_canonical_mps(self.bonds, seed)
        self.eng = Engine(self.mpo, device=device, t_budget_bytes=t_budget_bytes)
        self.eng.init_boundaries()
        K = self.K
        for k in range(K - 1, 1, -1):
            self.eng.update_right(k, self.bonds[k], self.bonds[k + 1],
                                  site_payload(self.bonds[k], self.bonds[k + 1], self.tensors[k], device))
        self.center = None      # one-site center tensor after a split
        self.center_site = None
        self.log = []

    def _grad_step(self, i, psi0):
        """Adjoint at sites (i, i+1) with cotangent psi: d<psi|H_eff|psi>/dW for the
        two site tensors of the MPO (each half of the symmetric derivative)."""
        import torch
        bl, br = self.bonds[i], self.bonds[i + 2]
        Lb, Rb = X.Bond(bl), X.Bond(br)
        L, R = self.eng.left[i], self.eng.right[i + 2]
        vjp = self.eng.vjp_plan(i, bl, br)
        psi = torch.from_numpy(X.pack_psi(Lb, Rb, psi0)).to(self.device)
        X.normalize(psi, self._gws)
        f64 = dict(dtype=torch.float64, device=self.device)
        g_psi = torch.empty_like(psi)
        g_L, g_R = torch.empty(max(L.numel(), 1), **f64), torch.empty(max(R.numel(), 1), **f64)
        g_w1 = torch.empty(max(16 * vjp.nnz1, 1), **f64)
        g_w2 = torch.empty(max(16 * vjp.nnz2, 1), **f64)
        vjp.prepare(L, R)
        vjp.backward(L, R, psi, psi, g_psi, g_L, g_R, g_w1, g_w2)
        # with cotangent psi the W parts of the VJP are d<psi|H_eff|psi>/dW at fixed psi,
        # and g_psi = H_eff^T psi gives E = <psi, g_psi>
        energy = float(torch.dot(psi, g_psi))
        for site, gw, nnz in ((i, g_w1, vjp.nnz1), (i + 1, g_w2, vjp.nnz2)):
            if site not in self._wgrad:
                self._wgrad[site] = gw[:16 * nnz].view(nnz, 4, 4).cpu().numpy()
        self.log.append({"pass": "grad", "i": i, "energy": energy})
        return psi0

    def mpo_gradients(self):
        """dE/d(MPO values) of E = <MPS|H|MPS> for the current, normalised MPS.

        E depends on the values of site k's MPO tensor only through the two-site
        H_eff of any pair containing k, so one pass that moves the two-site centre
        over the chain (splitting without truncation: the bond ranks never exceed M
        after a sweep) and takes the adjoint of the sigma-vector with cotangent psi
        at each pair gives every site's gradient.  Must follow a right-to-left pass
        (centre at sites 0, 1).  Returns a list over sites of (nnz, 4, 4) arrays
        aligned with mpo.sites[k] entries."""
        import torch
        if self.center_site != 1:
            raise RuntimeError("mpo_gradients: run an even number of passes first (centre at sites 0, 1)")
        self._wgrad = {}
        self._gws = torch.zeros(max(X.davidson_ws_bytes(1, 1) // 8, 1), dtype=torch.float64, device=self.device)
        K = self.K
        psi0 = contract_two(self.tensors[0], self.center, self.bonds[0], self.bonds[1], self.bonds[2])
        for i in range(0, K - 1):
            if i > 0:
                psi0 = contract_two(self.center, self.tensors[i + 1], self.bonds[i], self.bonds[i + 1],
                                    self.bonds[i + 2])
            psi = self._grad_step(i, psi0)
            if i < K - 2:
                nb, A, C, _ = split(psi, self.bonds[i], self.bonds[i + 2], self.M, 0)
                self.bonds[i + 1] = nb
                self.tensors[i] = A
                self.center, self.center_site = C, i + 1
                self.eng.update_left(i, self.bonds[i], self.bonds[i + 1],
                                     site_payload(self.bonds[i], self.bonds[i + 1], A, self.device))
            else:
                nb, B, C, _ = split(psi, self.bonds[i], self.bonds[i + 2], self.M, 1)
                self.bonds[i + 1] = nb
                self.tensors[i + 1] = B
                self.center, self.center_site = C, i
                self.eng.update_right(i + 1, self.bonds[i + 1], self.bonds[i + 2],
                                      site_payload(self.bonds[i + 1], self.bonds[i + 2], B, self.device))
        return [self._wgrad[k] for k in range(K)]

    def _mpo(self, h, g):
        return build_mpo(h, g, switch=self.mpo_switch)

    def integral_derivative(self, wgrad, dh, dg):
        """Directional derivative dE/dt of E(h + t dh, g + t dg) at fixed MPS from the
        MPO-value gradients: the MPO values are affine in the integrals, so the
        change of every value along (dh, dg) is (W(h + dh) - W(h - dh)) / 2 exactly."""
        plus = self._mpo(self.h + dh, self.g + dg)
        minus = self._mpo(self.h - dh, self.g - dg)
        total = 0.0
        for k in range(self.K):
            sp, sm, s0 = plus.sites[k], minus.sites[k], self.mpo.sites[k]
            if not (np.array_equal(sp.rows, s0.rows) and np.array_equal(sp.cols, s0.cols)
                    and np.array_equal(sm.rows, s0.rows) and np.array_equal(sm.cols, s0.cols)):
                raise RuntimeError("integral_derivative: MPO structure changed along the direction")
            dW = 0.5 * (np.asarray(sp.mats).reshape(-1, 4, 4) - np.asarray(sm.mats).reshape(-1, 4, 4))
            total += float(np.sum(wgrad[k] * dW))
        return total

    def one_rdm(self, wgrad):
        """Spin-summed 1-RDM gamma_pq = <sum_s a+_ps a_qs> of the current MPS as the
        integral gradient dE/dh (symmetric directions: e_pp, and e_pq + e_qp which
        gives gamma_pq + gamma_qp = 2 gamma_pq)."""
        K = self.K
        gam = np.zeros((K, K))
        zg = np.zeros_like(self.g)
        for p in range(K):
            for q in range(p, K):
                dh = np.zeros((K, K))
                dh[p, q] = dh[q, p] = 1.0
                d = self.integral_derivative(wgrad, dh, zg)
                gam[p, q] = gam[q, p] = d if p == q else 0.5 * d
        return gam

    def two_rdm(self, wgrad):
        """Spin-summed 2-RDM Gamma_pqrs = <sum_st a+_ps a+_rt a_st a_qs> of the current
        MPS, symmetrised over the eight index permutations that leave (pq|rs)
        integrals unchanged -- the part the energy sees, E = sum h gamma + 1/2 sum g
        Gamma (Sec. II.E.1).  For each permutation orbit O, the direction dg = 1 on O
        gives dE/dt = 1/2 sum_O Gamma; the MPO values are affine in g, so their change
        along dg is W(g + dg) - W(g) exactly.  One MPO construction per orbit (about
        K^4 / 8): meant for small active spaces."""
        K = self.K
        base = [np.asarray(self.mpo.sites[k].mats).reshape(-1, 4, 4) for k in range(K)]
        pairs = [(p, q) for p in range(K) for q in range(p + 1)]
        gam2 = np.zeros((K, K, K, K))
        for a in range(len(pairs)):
            for b in range(a + 1):
                (p, q), (r, s) = pairs[a], pairs[b]
                orbit = {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                         (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}
                dg = np.zeros_like(self.g)
                for x in orbit:
                    dg[x] = 1.0
                plus = self._mpo(self.h, self.g + dg)
                d = 0.0
                for k in range(K):
                    sp, s0 = plus.sites[k], self.mpo.sites[k]
                    if not (np.array_equal(sp.rows, s0.rows) and np.array_equal(sp.cols, s0.cols)):
                        raise RuntimeError("two_rdm: MPO structure changed along a direction")
                    d += float(np.sum(wgrad[k] * (np.asarray(sp.mats).reshape(-1, 4, 4) - base[k])))
                val = 2.0 * d / len(orbit)
                for x in orbit:
                    gam2[x] = val
        return gam2

    def _step(self, i, psi0, pass_id):
        import torch
        t0 = time.perf_counter()
        bl, br = self.bonds[i], self.bonds[i + 2]
        plan = self.eng.heff_plan(i, bl, br)
        t1 = time.perf_counter()
        Lb, Rb = X.Bond(bl), X.Bond(br)
        L, R = self.eng.left[i], self.eng.right[i + 2]
        n = int(plan.info.psi_nnz)
        psi_t = torch.from_numpy(X.pack_psi(Lb, Rb, psi0)).to(self.device)
        diag = torch.empty(n, dtype=torch.float64, device=self.device)
        plan.prepare(L, R)
        plan.diag(L, R, diag)
        dav = Davidson(n, min(self.kmax, max(n, 1)), self.device)

        def mv(v, out):
            plan.apply(L, R, v, out)

        if self.precision != "f64":
            plan.lower_f32(L, R)
            v32 = torch.empty(n, dtype=torch.float32, device=self.device)
            s32 = torch.empty(n, dtype=torch.float32, device=self.device)
            low = plan.apply_bf16 if self.precision == "bf16" else plan.apply_f32

            def mv32(v, out):
                X.convert_f64_f32(v, v32)
                low(v32, s32)
                X.convert_f32_f64(s32, out)

            theta, rnorm, n32, n64 = dav.solve_mixed(mv32, mv, psi_t, diag, tol=self.tol, max_iter=self.max_iter,
                                                     **PRECISIONS[self.precision])
            nmv = n32 + n64
        else:
            theta, rnorm, nmv = dav.solve(mv, psi_t, diag, tol=self.tol, max_iter=self.max_iter)
        psi = X.unpack_psi(Lb, Rb, dav.x.cpu().numpy())
        # the plan stays cached for the site; its workspace (mixed and stacked
        # operators, intermediates) is only needed during the step
        plan.release_workspace()
        self.log.append({"pass": pass_id, "i": i, "energy": theta, "rnorm": rnorm, "n_matvec": nmv,
                         "sigma_flop": float(plan.info.flops_useful),
                         "t_plan": t1 - t0, "t_solve": time.perf_counter() - t1})
        return psi

    def _split_logged(self, psi, i, direction):
        """Truncating split of the step's Ritz vector; the step's log record gets the
        discarded weight, the new middle bond and its kept singular values."""
        info = {}
        nb, canon, centre, disc = split(psi, self.bonds[i], self.bonds[i + 2], self.M, direction, info=info)
        self.log[-1].update(discarded=disc, bond=list(nb), kept_s=info["kept_s"])
        return nb, canon, centre

    def _timed(self, key, t0):
        """Host wall time since t0 into the step's log record (GPU work is
        asynchronous: an environment update shows up in the next step's solve)."""
        t = time.perf_counter()
        self.log[-1][key] = self.log[-1].get(key, 0.0) + t - t0
        return t

    def sweep_left_to_right(self, pass_id, start):
        K = self.K
        for i in range(start, K - 1):
            t0 = time.perf_counter()
            if i == 0 and self.center is None:
                psi0 = contract_two(self.tensors[0], self.tensors[1], self.bonds[0], self.bonds[1], self.bonds[2])
            else:
                psi0 = contract_two(self.center, self.tensors[i + 1], self.bonds[i], self.bonds[i + 1],
                                    self.bonds[i + 2])
            tc = time.perf_counter() - t0
            psi = self._step(i, psi0, pass_id)
            self.log[-1]["t_contract"] = tc
            t0 = time.perf_counter()
            if i < K - 2:
                nb, A, C = self._split_logged(psi, i, 0)
                self.bonds[i + 1] = nb
                self.eng.prefetch_env_plan(0, i, self.bonds[i], self.bonds[i + 1])
                self.eng.prefetch_heff_plan(i + 1, self.bonds[i + 1], self.bonds[i + 3])
                self.tensors[i] = A
                self.center, self.center_site = C, i + 1
                t0 = self._timed("t_split", t0)
                self.eng.update_left(i, self.bonds[i], self.bonds[i + 1],
                                     site_payload(self.bonds[i], self.bonds[i + 1], A, self.device))
            else:
                nb, B, C = self._split_logged(psi, i, 1)
                self.bonds[i + 1] = nb
                self.tensors[i + 1] = B
                self.center, self.center_site = C, i
                t0 = self._timed("t_split", t0)
                self.eng.update_right(i + 1, self.bonds[i + 1], self.bonds[i + 2],
                                      site_payload(self.bonds[i + 1], self.bonds[i + 2], B, self.device))
            self._timed("t_env", t0)

    def sweep_right_to_left(self, pass_id):
        for i in range(self.K - 3, -1, -1):
            t0 = time.perf_counter()
            psi0 = contract_two(self.tensors[i], self.center, self.bonds[i], self.bonds[i + 1], self.bonds[i + 2])
            tc = time.perf_counter() - t0
            psi = self._step(i, psi0, pass_id)
            self.log[-1]["t_contract"] = tc
            t0 = time.perf_counter()
            if i > 0:
                nb, B, C = self._split_logged(psi, i, 1)
                self.bonds[i + 1] = nb
                self.eng.prefetch_env_plan(1, i + 1, self.bonds[i + 1], self.bonds[i + 2])
                self.eng.prefetch_heff_plan(i - 1, self.bonds[i - 1], self.bonds[i + 1])
                self.tensors[i + 1] = B
                self.center, self.center_site = C, i
                t0 = self._timed("t_split", t0)
                self.eng.update_right(i + 1, self.bonds[i + 1], self.bonds[i + 2],
                                      site_payload(self.bonds[i + 1], self.bonds[i + 2], B, self.device))
            else:
                nb, A, C = self._split_logged(psi, i, 0)
                self.bonds[i + 1] = nb
                self.tensors[i] = A
                self.center, self.center_site = C, i + 1
                t0 = self._timed("t_split", t0)
                self.eng.update_left(i, self.bonds[i], self.bonds[i + 1],
                                     site_payload(self.bonds[i], self.bonds[i + 1], A, self.device))
            self._timed("t_env", t0)

    # -- one-site passes (Sec. II.A.2): the bond spaces are the ones the two-site
    # passes chose; each step solves the one-site H_eff and moves the centre with an
    # SVD that keeps every sector's dimension.
    def _step1(self, i, pass_id):
        import torch
        bl, br = self.bonds[i], self.bonds[i + 1]
        plan = self.eng.heff1_plan(i, bl, br)
        Lb, Rb = X.Bond(bl), X.Bond(br)
        L, R = self.eng.left[i], self.eng.right[i + 1]
        n = int(plan.info.psi_nnz)
        psi_t = torch.from_numpy(X.pack_psi1(Lb, Rb, self.center)).to(self.device)
        diag = torch.empty(n, dtype=torch.float64, device=self.device)
        plan.prepare(L, R)
        plan.diag(L, R, diag)
        dav = Davidson(n, min(self.kmax, max(n, 1)), self.device)

        def mv(v, out):
            plan.apply(L, R, v, out)

        theta, rnorm, nmv = dav.solve(mv, psi_t, diag, tol=self.tol, max_iter=self.max_iter)
        self.center = X.unpack_psi1(Lb, Rb, dav.x.cpu().numpy())
        plan.release_workspace()
        self.log.append({"pass": pass_id, "i": i, "one_site": True, "energy": theta, "rnorm": rnorm,
                         "n_matvec": nmv})
        return theta

    def _move1(self, i, direction):
        """Move the one-site centre from site i to i+1 (direction 0) or i-1 (1)."""
        if direction == 0:
            psi2 = {(il, s, 0, ir): b for (il, s, ir), b in self.center.items()}
            fixed = {tuple(q): m for q, m in self.bonds[i + 1]}
            nb, A, F, _ = split(psi2, self.bonds[i], self.bonds[i + 1], self.M, 0, fixed=fixed)
            self.bonds[i + 1] = nb
            self.tensors[i] = A
            self.eng.update_left(i, self.bonds[i], self.bonds[i + 1],
                                 site_payload(self.bonds[i], self.bonds[i + 1], A, self.device))
            by_l = {}
            for (ir, s, ir2), b in self.tensors[i + 1].items():
                by_l.setdefault(ir, []).append((s, ir2, b))
            c = {}
            for (q, _, ir), f in F.items():
                for s, ir2, b in by_l.get(ir, []):
                    key = (q, s, ir2)
                    c[key] = c[key] + f @ b if key in c else f @ b
            self.center, self.center_site = c, i + 1
        else:
            psi2 = {(il, 0, s, ir): b for (il, s, ir), b in self.center.items()}
            fixed = {tuple(q): m for q, m in self.bonds[i]}
            nb, B, F, _ = split(psi2, self.bonds[i], self.bonds[i + 1], self.M, 1, fixed=fixed)
            self.bonds[i] = nb
            self.tensors[i] = B
            self.eng.update_right(i, self.bonds[i], self.bonds[i + 1],
                                  site_payload(self.bonds[i], self.bonds[i + 1], B, self.device))
            by_r = {}
            for (il, _, q), f in F.items():
                by_r.setdefault(il, []).append((q, f))
            c = {}
            for (il2, s, il), a in self.tensors[i - 1].items():
                for q, f in by_r.get(il, []):
                    key = (il2, s, q)
                    c[key] = c[key] + a @ f if key in c else a @ f
            self.center, self.center_site = c, i - 1

    def run_one_site(self, n_passes):
        """Alternating one-site passes from the current centre (after an even number
        of two-site passes: centre at site 1); returns the last energy of each pass."""
        if self.center_site is None:
            raise RuntimeError("run_one_site: run two-site passes first (they fix the bond spaces)")
        out = []
        for p in range(n_passes):
            if p % 2 == 0:
                for i in range(self.center_site, self.K):
                    self._step1(i, ("one", p))
                    if i < self.K - 1:
                        self._move1(i, 0)
            else:
                for i in range(self.center_site, -1, -1):
                    self._step1(i, ("one", p))
                    if i > 0:
                        self._move1(i, 1)
            out.append(self.log[-1]["energy"])
        return out

    def run(self, n_sweeps):
        """Alternating passes; returns the energy of the last step of each pass."""
        out = []
        for s in range(n_sweeps):
            if s % 2 == 0:
                self.sweep_left_to_right(s, 0 if s == 0 else 1)
            else:
                self.sweep_right_to_left(s)
            out.append(self.log[-1]["energy"])
        return out
