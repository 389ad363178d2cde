"""ctypes binding of libheffx.so (argument marshalling only).

Every computation runs in the HIP library; this module converts numpy tables to
the C structs of include/heffx.h, hands over device pointers of torch tensors
and the current HIP stream, and checks return codes.  If the library is missing
the import of any entry point raises: there is no fallback path.
"""

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libheffx.so")

HX_OK, HX_EINVAL, HX_EHIP, HX_EUNSUP = 0, -1, -2, -3

EXPORTED = (
    "hx_env_layout", "hx_psi_layout", "hx_site_layout", "hx_heff_plan_create", "hx_env_plan_create",
    "hx_plan_get_info", "hx_plan_upload", "hx_plan_destroy", "hx_heff_prepare", "hx_heff_apply",
    "hx_heff_diag", "hx_env_update", "hx_davidson_ws_bytes", "hx_davidson_step", "hx_dots",
    "hx_normalize", "hx_convert_f64_f32", "hx_convert_f32_f64", "hx_heff_lower_f32", "hx_heff_apply_f32",
    "hx_heff_plan_batch", "hx_batch_offsets", "hx_heff_graph_create", "hx_graph_launch", "hx_graph_destroy",
    "hx_heff_vjp_plan_create", "hx_heff_apply_backward", "hx_heff_apply_bf16", "hx_davidson_restart2",
    "hx_heff1_plan_create", "hx_psi1_layout", "hx_heff1_vjp_plan_create", "hx_gather_index",
    "hx_scatter_index", "hx_axpy", "hx_heff_apply_backward_f32", "hx_heff_apply_noalloc",
    "hx_last_error",
)


class HxBond(ctypes.Structure):
    _fields_ = [("nsec", c_int32), ("qn", POINTER(c_int32)), ("dim", POINTER(c_int32))]


class HxOpset(ctypes.Structure):
    _fields_ = [("nop", c_int32), ("dq", POINTER(c_int32))]


class HxMpoSite(ctypes.Structure):
    _fields_ = [("nnz", c_int64), ("row", POINTER(c_int32)), ("col", POINTER(c_int32)),
                ("val", POINTER(c_double))]


class HxPlanOpts(ctypes.Structure):
    _fields_ = [("t_budget_bytes", c_int64), ("split_kseg_min", c_int32), ("kernel_variant", c_int32),
                ("n_roots", c_int32), ("b_part", c_int32), ("b_nparts", c_int32), ("t_merge_off", c_int32),
                ("reserved", c_int32 * 2)]


class HxPlanInfo(ctypes.Structure):
    _fields_ = [("psi_nnz", c_int64), ("in_nnz", c_int64), ("in2_nnz", c_int64), ("out_nnz", c_int64),
                ("table_bytes", c_int64), ("ws_bytes", c_int64), ("flops_apply", c_double),
                ("flops_prepare", c_double), ("bytes_apply", c_double), ("n_tasks", c_int64),
                ("n_tiles", c_int64), ("n_chunks", c_int32), ("n_mixed", c_int32), ("flops_useful", c_double)]


_lib = None


def lib():
    """Load libheffx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"heffx HIP library not built: {LIB_PATH} missing "
                           "(run __graft_entry__.build() or python paper_2310_03920_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.hx_last_error.restype = ctypes.c_char_p
    L.hx_env_layout.argtypes = [P(HxBond), P(HxOpset), P(c_int64), P(c_int64)]
    L.hx_psi_layout.argtypes = [P(HxBond), P(HxBond), c_int64, P(c_int32), P(c_int64)]
    L.hx_psi_layout.restype = c_int64
    L.hx_site_layout.argtypes = [P(HxBond), P(HxBond), c_int64, P(c_int32), P(c_int64)]
    L.hx_site_layout.restype = c_int64
    L.hx_heff_plan_create.argtypes = [P(HxBond), P(HxBond), P(HxOpset), P(HxOpset), P(HxOpset),
                                      P(HxMpoSite), P(HxMpoSite), P(HxPlanOpts), P(c_void_p)]
    L.hx_env_plan_create.argtypes = [c_int, P(HxBond), P(HxBond), P(HxOpset), P(HxOpset), P(HxMpoSite),
                                     P(HxPlanOpts), P(c_void_p)]
    L.hx_plan_get_info.argtypes = [c_void_p, P(HxPlanInfo)]
    L.hx_plan_upload.argtypes = [c_void_p, c_void_p, c_void_p]
    L.hx_plan_destroy.argtypes = [c_void_p]
    L.hx_plan_destroy.restype = None
    L.hx_heff_prepare.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_heff_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_heff_diag.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_heff_apply_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_env_update.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_davidson_ws_bytes.argtypes = [c_int64, c_int32]
    L.hx_davidson_ws_bytes.restype = c_int64
    L.hx_davidson_step.argtypes = [c_int64, c_int32, c_int32, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                   c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_dots.argtypes = [c_int64, c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_normalize.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hx_convert_f64_f32.argtypes = [c_int64, c_void_p, c_void_p, c_void_p]
    L.hx_convert_f32_f64.argtypes = [c_int64, c_void_p, c_void_p, c_void_p]
    L.hx_heff_lower_f32.argtypes = [c_void_p] + [c_void_p] * 7
    L.hx_heff_apply_f32.argtypes = [c_void_p] + [c_void_p] * 6
    L.hx_heff_apply_bf16.argtypes = [c_void_p] + [c_void_p] * 6
    L.hx_davidson_restart2.argtypes = [c_int64] + [c_void_p] * 9
    L.hx_heff_plan_batch.argtypes = [P(c_void_p), c_int32, P(c_void_p)]
    L.hx_batch_offsets.argtypes = [c_void_p, c_int32, P(c_int64), P(c_int64), P(c_int64)]
    L.hx_heff_vjp_plan_create.argtypes = L.hx_heff_plan_create.argtypes
    L.hx_heff1_plan_create.argtypes = [P(HxBond), P(HxBond), P(HxOpset), P(HxOpset), P(HxMpoSite), P(HxPlanOpts),
                                       P(c_void_p)]
    L.hx_heff1_vjp_plan_create.argtypes = L.hx_heff1_plan_create.argtypes
    L.hx_gather_index.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.hx_scatter_index.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.hx_axpy.argtypes = [c_int64, ctypes.c_double, c_void_p, c_void_p, c_void_p]
    L.hx_heff_apply_backward_f32.argtypes = [c_void_p] + [c_void_p] * 11
    L.hx_psi1_layout.argtypes = [P(HxBond), P(HxBond), c_int64, P(c_int32), P(c_int64)]
    L.hx_psi1_layout.restype = c_int64
    L.hx_heff_apply_backward.argtypes = [c_void_p] * 11 + [c_void_p]
    L.hx_heff_graph_create.argtypes = [c_void_p, c_int32] + [c_void_p] * 5 + [P(c_void_p)]
    L.hx_graph_launch.argtypes = [c_void_p, c_void_p]
    L.hx_graph_destroy.argtypes = [c_void_p]
    L.hx_graph_destroy.restype = None
    _lib = L
    return L


def check(rc, what):
    if rc != HX_OK:
        msg = lib().hx_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed (code {rc}): {msg}")


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Bond:
    """Sector table of one bond (list of ((N, 2Sz), dim), sorted)."""

    def __init__(self, sectors):
        self.sectors = [(tuple(q), int(m)) for q, m in sectors]
        self.qn = _i32([q for q, _ in self.sectors]).reshape(-1, 2)
        self.dim = _i32([m for _, m in self.sectors])
        self.c = HxBond(len(self.sectors), self.qn.ctypes.data_as(POINTER(c_int32)),
                        self.dim.ctypes.data_as(POINTER(c_int32)))
        self.index = {q: i for i, (q, _) in enumerate(self.sectors)}

    @property
    def nsec(self):
        return len(self.sectors)


class OpSet:
    def __init__(self, dq):
        self.dq = _i32(dq).reshape(-1, 2)
        self.c = HxOpset(self.dq.shape[0], self.dq.ctypes.data_as(POINTER(c_int32)))

    @property
    def nop(self):
        return self.dq.shape[0]


class MpoSite:
    def __init__(self, rows, cols, mats):
        self.rows = _i32(rows)
        self.cols = _i32(cols)
        self.vals = np.ascontiguousarray(np.asarray(mats, dtype=np.float64).reshape(-1, 16))
        self.c = HxMpoSite(len(self.rows), self.rows.ctypes.data_as(POINTER(c_int32)),
                           self.cols.ctypes.data_as(POINTER(c_int32)),
                           self.vals.ctypes.data_as(POINTER(c_double)))

    @classmethod
    def from_entries(cls, entries):
        if not entries:
            return cls(np.zeros(0), np.zeros(0), np.zeros((0, 16)))
        return cls([e[0] for e in entries], [e[1] for e in entries], [e[2] for e in entries])


def env_layout(bond, ops):
    op_off = np.zeros(ops.nop + 1, np.int64)
    blk_off = np.zeros(max(ops.nop * bond.nsec, 1), np.int64)
    check(lib().hx_env_layout(ctypes.byref(bond.c), ctypes.byref(ops.c),
                              op_off.ctypes.data_as(POINTER(c_int64)), blk_off.ctypes.data_as(POINTER(c_int64))),
          "env_layout")
    return op_off, blk_off[:ops.nop * bond.nsec].reshape(ops.nop, bond.nsec)


def psi_layout(lbond, rbond):
    n = lib().hx_psi_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), 0, None, None)
    if n < 0:
        check(int(n), "psi_layout")
    keys = np.zeros((max(n, 1), 4), np.int32)
    off = np.zeros(n + 1, np.int64)
    n2 = lib().hx_psi_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), n,
                             keys.ctypes.data_as(POINTER(c_int32)), off.ctypes.data_as(POINTER(c_int64)))
    if n2 < 0:
        check(int(n2), "psi_layout")
    return [tuple(int(x) for x in k) for k in keys[:n]], off


def psi1_layout(lbond, rbond):
    n = lib().hx_psi1_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), 0, None, None)
    if n < 0:
        check(int(n), "psi1_layout")
    keys = np.zeros((max(n, 1), 3), np.int32)
    off = np.zeros(n + 1, np.int64)
    n2 = lib().hx_psi1_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), n,
                              keys.ctypes.data_as(POINTER(c_int32)), off.ctypes.data_as(POINTER(c_int64)))
    if n2 < 0:
        check(int(n2), "psi1_layout")
    return [tuple(int(x) for x in k) for k in keys[:n]], off


def pack_psi1(lbond, rbond, t):
    """One-site tensor {(il, s, ir): block} -> flat payload in the one-site layout."""
    keys, off = psi1_layout(lbond, rbond)
    out = np.zeros(int(off[-1]))
    for i, k in enumerate(keys):
        if k in t:
            out[off[i]:off[i + 1]] = t[k].ravel()
    return out


def unpack_psi1(lbond, rbond, flat):
    keys, off = psi1_layout(lbond, rbond)
    res = {}
    for i, (il, s, ir) in enumerate(keys):
        res[(il, s, ir)] = np.asarray(flat[off[i]:off[i + 1]]).reshape(lbond.sectors[il][1],
                                                                      rbond.sectors[ir][1]).copy()
    return res


def site_layout(lbond, rbond):
    n = lib().hx_site_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), 0, None, None)
    if n < 0:
        check(int(n), "site_layout")
    keys = np.zeros((max(n, 1), 3), np.int32)
    off = np.zeros(n + 1, np.int64)
    n2 = lib().hx_site_layout(ctypes.byref(lbond.c), ctypes.byref(rbond.c), n,
                              keys.ctypes.data_as(POINTER(c_int32)), off.ctypes.data_as(POINTER(c_int64)))
    if n2 < 0:
        check(int(n2), "site_layout")
    return [tuple(int(x) for x in k) for k in keys[:n]], off


def site_to_psi1_index(lbond, rbond):
    """Element permutation between a site tensor's payload (hx_site_layout) and the
    same tensor in the one-site wavefunction layout (hx_psi1_layout): psi1[j] =
    site[idx[j]].  Both layouts hold the same blocks (il, s, ir), row-major."""
    skeys, soff = site_layout(lbond, rbond)
    pkeys, poff = psi1_layout(lbond, rbond)
    where = {k: int(soff[i]) for i, k in enumerate(skeys)}
    idx = np.empty(int(poff[-1]), np.int64)
    for i, k in enumerate(pkeys):
        n = int(poff[i + 1] - poff[i])
        idx[poff[i]:poff[i + 1]] = where[k] + np.arange(n)
    return idx


# ------------------------------------------------------------------ packing (host data marshalling)

def pack_env(bond, ops_dq, env):
    """Environment in block-dict form -> flat payload in the library layout."""
    ops = OpSet(ops_dq)
    op_off, blk_off = env_layout(bond, ops)
    out = np.zeros(int(op_off[-1]))
    for a, op in enumerate(env):
        for isrc, blk in op["blocks"].items():
            o = blk_off[a, isrc]
            if o < 0:
                raise ValueError("block outside the operator's shift")
            out[o:o + blk.size] = blk.ravel()
    return out


def unpack_env(bond, ops_dq, flat):
    ops = OpSet(ops_dq)
    op_off, blk_off = env_layout(bond, ops)
    res = []
    for a in range(ops.nop):
        dq = tuple(int(x) for x in ops.dq[a])
        blocks = {}
        for isrc in range(bond.nsec):
            o = blk_off[a, isrc]
            if o < 0:
                continue
            q = bond.sectors[isrc][0]
            idst = bond.index[(q[0] + dq[0], q[1] + dq[1])]
            m, n = bond.sectors[idst][1], bond.sectors[isrc][1]
            blocks[isrc] = np.asarray(flat[o:o + m * n]).reshape(m, n).copy()
        res.append({"dq": dq, "blocks": blocks})
    return res


def pack_roots(lbond, rbond, flats):
    """R single-root payloads -> the multi-root layout (roots side by side per column block)."""
    keys, off = psi_layout(lbond, rbond)
    R = len(flats)
    out = np.zeros(int(off[-1]) * R)
    cols = {}
    for i, (il, s1, s2, ir) in enumerate(keys):
        cols.setdefault((s2, ir), []).append(i)
    for (s2, ir), idx in cols.items():
        dr = rbond.sectors[ir][1]
        a, b = int(off[idx[0]]), int(off[idx[-1] + 1])
        rows = (b - a) // dr
        blk = np.stack([np.asarray(f[a:b]).reshape(rows, dr) for f in flats], axis=1)  # rows x R x dr
        out[R * a:R * b] = blk.ravel()
    return out


def unpack_roots(lbond, rbond, flat, R):
    keys, off = psi_layout(lbond, rbond)
    outs = [np.zeros(int(off[-1])) for _ in range(R)]
    cols = {}
    for i, (il, s1, s2, ir) in enumerate(keys):
        cols.setdefault((s2, ir), []).append(i)
    for (s2, ir), idx in cols.items():
        dr = rbond.sectors[ir][1]
        a, b = int(off[idx[0]]), int(off[idx[-1] + 1])
        rows = (b - a) // dr
        blk = np.asarray(flat[R * a:R * b]).reshape(rows, R, dr)
        for rho in range(R):
            outs[rho][a:b] = blk[:, rho, :].ravel()
    return outs


def pack_psi(lbond, rbond, psi):
    keys, off = psi_layout(lbond, rbond)
    out = np.zeros(int(off[-1]))
    for i, k in enumerate(keys):
        if k in psi:
            out[off[i]:off[i + 1]] = psi[k].ravel()
    return out


def unpack_psi(lbond, rbond, flat):
    keys, off = psi_layout(lbond, rbond)
    res = {}
    for i, (il, s1, s2, ir) in enumerate(keys):
        res[(il, s1, s2, ir)] = np.asarray(flat[off[i]:off[i + 1]]).reshape(lbond.sectors[il][1],
                                                                          rbond.sectors[ir][1]).copy()
    return res


def pack_site(lbond, rbond, t):
    keys, off = site_layout(lbond, rbond)
    out = np.zeros(int(off[-1]))
    for i, k in enumerate(keys):
        if k in t:
            out[off[i]:off[i + 1]] = t[k].ravel()
    return out


def unpack_site(lbond, rbond, flat):
    keys, off = site_layout(lbond, rbond)
    res = {}
    for i, (il, s, ir) in enumerate(keys):
        res[(il, s, ir)] = np.asarray(flat[off[i]:off[i + 1]]).reshape(lbond.sectors[il][1],
                                                                      rbond.sectors[ir][1]).copy()
    return res


# ------------------------------------------------------------------ plans

def _ptr(t):
    return c_void_p(0) if t is None else c_void_p(t.data_ptr())


def need_all(device, *items):
    """need() over (tensor, name, n, dtype) items: every operand's type, dtype,
    layout and length first, then where they live."""
    for t, name, n, dt in items:
        need(t, name, n, dt, device, where=False)
    for t, name, n, dt in items:
        need(t, name, n, dt, device)


def need(t, name, n, dtype="float64", device=None, where=True):
    """Check a device operand before its pointer reaches the library, whose entry
    points take bare pointers with lengths implied by the plan: a torch tensor of
    the given dtype, contiguous, with at least n elements and (with `where`) on
    the plan's GPU.  A missing operand (None) is accepted only when n == 0.
    Raises TypeError / ValueError; no device work is issued."""
    import torch
    if t is None:
        if n == 0:
            return
        raise ValueError(f"{name}: missing (the plan needs {n} elements)")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = getattr(torch, dtype)
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} elements, the plan needs {n}")
    if where and (not t.is_cuda or (device is not None and t.device != device)):
        raise ValueError(f"{name}: must be a tensor on the plan's device ({device or 'a GPU'}), got {t.device}")


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A host plan; `upload(device)` places its tables and a workspace on the GPU."""

    def __init__(self, handle, keep):
        self.h = handle
        self._keep = keep
        info = HxPlanInfo()
        check(lib().hx_plan_get_info(self.h, ctypes.byref(info)), "plan_get_info")
        self.info = info
        self.tables = None
        self.ws = None
        self._ready = False

    def upload(self, device="cuda"):
        import torch
        nb = int(self.info.table_bytes) + 256
        buf = torch.empty(nb, dtype=torch.uint8, device=device)
        shift = (-buf.data_ptr()) % 256
        self.tables = buf
        self._tab_ptr = buf.data_ptr() + shift
        check(lib().hx_plan_upload(self.h, c_void_p(self._tab_ptr), _stream()), "plan_upload")
        nws = max(int(self.info.ws_bytes) // 8, 1)
        self.ws = torch.empty(nws, dtype=torch.float64, device=device)
        self._ready = False
        return self

    def release_workspace(self):
        """Free the device workspace and the FP32 copies; the tables stay on the
        device.  prepare() needs ensure_workspace() first."""
        self.ws = None
        self.ws32 = self.L32 = self.R32 = None
        self._ready = False

    def ensure_workspace(self):
        """Allocate the workspace again after release_workspace()."""
        import torch
        if self.ws is None and self.tables is not None:
            nws = max(int(self.info.ws_bytes) // 8, 1)
            self.ws = torch.empty(nws, dtype=torch.float64, device=self.tables.device)
            self._ready = False
        return self

    @property
    def device(self):
        return None if self.ws is None else self.ws.device

    def _uploaded(self, what):
        if self.ws is None or self.tables is None:
            raise RuntimeError(f"{what}: upload the plan to a device first")

    def _prepared(self, what):
        """Sigma-vector, diagonal and adjoint calls read the mixed operators that
        prepare() leaves in the workspace."""
        self._uploaded(what)
        if not self._ready:
            raise RuntimeError(f"{what}: call prepare(L, R) first")

    def _lowered(self, what):
        if getattr(self, "L32", None) is None:
            raise RuntimeError(f"{what}: call lower_f32 first")

    def _env_items(self, L, R, dtype="float64"):
        return [(L, "L", int(self.info.in_nnz), dtype), (R, "R", int(self.info.in2_nnz), dtype)]

    def _check_env(self, L, R, dtype="float64"):
        need_all(self.device, *self._env_items(L, R, dtype))

    def __del__(self):
        try:
            if self.h:
                lib().hx_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass


def _opts(t_budget_bytes=0, split_kseg_min=0, kernel_variant=0, n_roots=1, b_part=0, b_nparts=1, t_merge_off=0):
    o = HxPlanOpts()
    o.t_budget_bytes = int(t_budget_bytes)
    o.split_kseg_min = int(split_kseg_min)
    o.kernel_variant = int(kernel_variant)
    o.n_roots = int(n_roots)
    o.b_part = int(b_part)
    o.b_nparts = int(b_nparts)
    o.t_merge_off = int(bool(t_merge_off))
    return o


class HeffPlan(Plan):
    def __init__(self, lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, t_budget_bytes=0, split_kseg_min=0,
                 kernel_variant=0, n_roots=1, b_part=0, b_nparts=1, t_merge_off=0):
        lb, rb = (b if isinstance(b, Bond) else Bond(b) for b in (lbond, rbond))
        Lo, Mo, Ro = OpSet(Ldq), OpSet(mid_dq), OpSet(Rdq)
        w1 = W1 if isinstance(W1, MpoSite) else MpoSite.from_entries(W1)
        w2 = W2 if isinstance(W2, MpoSite) else MpoSite.from_entries(W2)
        opts = _opts(t_budget_bytes, split_kseg_min, kernel_variant, n_roots, b_part, b_nparts, t_merge_off)
        self.n_roots = int(n_roots)
        h = c_void_p()
        check(lib().hx_heff_plan_create(ctypes.byref(lb.c), ctypes.byref(rb.c), ctypes.byref(Lo.c),
                                        ctypes.byref(Mo.c), ctypes.byref(Ro.c), ctypes.byref(w1.c),
                                        ctypes.byref(w2.c), ctypes.byref(opts), ctypes.byref(h)),
              "heff_plan_create")
        super().__init__(h, (lb, rb, Lo, Mo, Ro, w1, w2))
        self.lbond, self.rbond = lb, rb

    def prepare(self, L, R):
        self._check_env(L, R)
        self._uploaded("heff_prepare")
        check(lib().hx_heff_prepare(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _stream()), "heff_prepare")
        self._ready = True

    def _check_vecs(self, psi, sigma, dtype="float64", env=()):
        n = int(self.info.psi_nnz)
        need_all(self.device, *env, (psi, "psi", n, dtype), (sigma, "sigma", n, dtype))
        if psi is not None and sigma is not None and n and psi.data_ptr() == sigma.data_ptr():
            raise ValueError("psi and sigma must not overlap")

    def apply(self, L, R, psi, sigma):
        self._check_vecs(psi, sigma, env=self._env_items(L, R))
        self._prepared("heff_apply")
        check(lib().hx_heff_apply(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _ptr(psi), _ptr(sigma), _stream()),
              "heff_apply")

    def apply_noalloc(self, L, R, psi, sigma):
        """prepare + apply with the library's static scratch array as workspace (no
        device allocation in the call; calls on one GPU must not overlap)."""
        self._check_vecs(psi, sigma, env=self._env_items(L, R))
        if self.tables is None:
            raise RuntimeError("heff_apply_noalloc: upload the plan to a device first")
        check(lib().hx_heff_apply_noalloc(self.h, _ptr(L), _ptr(R), _ptr(psi), _ptr(sigma), _stream()),
              "heff_apply_noalloc")

    def diag(self, L, R, out):
        nd = int(self.info.psi_nnz) // max(getattr(self, "n_roots", 1), 1)
        need_all(self.device, *self._env_items(L, R), (out, "diag", nd, "float64"))
        self._prepared("heff_diag")
        check(lib().hx_heff_diag(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _ptr(out), _stream()), "heff_diag")

    # FP32 mode: operands rounded once per (L, R); Davidson stays FP64
    def lower_f32(self, L, R):
        import torch
        self._check_env(L, R)
        self._prepared("heff_lower_f32")
        dev = self.ws.device
        if getattr(self, "ws32", None) is None:
            self.ws32 = torch.empty(max(int(self.info.ws_bytes) // 8, 1), dtype=torch.float32, device=dev)
        self.L32 = torch.empty(max(int(self.info.in_nnz), 1), dtype=torch.float32, device=dev)
        self.R32 = torch.empty(max(int(self.info.in2_nnz), 1), dtype=torch.float32, device=dev)
        check(lib().hx_heff_lower_f32(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _ptr(self.L32), _ptr(self.R32),
                                      _ptr(self.ws32), _stream()), "heff_lower_f32")

    def apply_f32(self, psi32, sigma32):
        self._check_vecs(psi32, sigma32, "float32")
        self._lowered("heff_apply_f32")
        check(lib().hx_heff_apply_f32(self.h, _ptr(self.L32), _ptr(self.R32), _ptr(self.ws32), _ptr(psi32),
                                      _ptr(sigma32), _stream()), "heff_apply_f32")

    def apply_bf16(self, psi32, sigma32):
        """BF16 block products on the FP32 operands of lower_f32."""
        self._check_vecs(psi32, sigma32, "float32")
        self._lowered("heff_apply_bf16")
        check(lib().hx_heff_apply_bf16(self.h, _ptr(self.L32), _ptr(self.R32), _ptr(self.ws32), _ptr(psi32),
                                       _ptr(sigma32), _stream()), "heff_apply_bf16")


class Heff1Plan(HeffPlan):
    """One-site sigma-vector plan (psi in the one-site layout)."""

    def __init__(self, lbond, rbond, Ldq, Rdq, W, t_budget_bytes=0, split_kseg_min=0, kernel_variant=0,
                 n_roots=1, t_merge_off=0):
        lb, rb = (b if isinstance(b, Bond) else Bond(b) for b in (lbond, rbond))
        Lo, Ro = OpSet(Ldq), OpSet(Rdq)
        w = W if isinstance(W, MpoSite) else MpoSite.from_entries(W)
        opts = _opts(t_budget_bytes, split_kseg_min, kernel_variant, n_roots, t_merge_off=t_merge_off)
        self.n_roots = int(n_roots)
        h = c_void_p()
        check(lib().hx_heff1_plan_create(ctypes.byref(lb.c), ctypes.byref(rb.c), ctypes.byref(Lo.c),
                                         ctypes.byref(Ro.c), ctypes.byref(w.c), ctypes.byref(opts),
                                         ctypes.byref(h)), "heff1_plan_create")
        Plan.__init__(self, h, (lb, rb, Lo, Ro, w))
        self.lbond, self.rbond = lb, rb


class HeffVjpPlan(Plan):
    """Plan of the vector-Jacobian products of sigma = H_eff psi."""

    def __init__(self, lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, t_budget_bytes=0, split_kseg_min=0,
                 kernel_variant=0):
        lb, rb = (b if isinstance(b, Bond) else Bond(b) for b in (lbond, rbond))
        Lo, Mo, Ro = OpSet(Ldq), OpSet(mid_dq), OpSet(Rdq)
        w1 = W1 if isinstance(W1, MpoSite) else MpoSite.from_entries(W1)
        w2 = W2 if isinstance(W2, MpoSite) else MpoSite.from_entries(W2)
        opts = _opts(t_budget_bytes, split_kseg_min, kernel_variant)
        h = c_void_p()
        check(lib().hx_heff_vjp_plan_create(ctypes.byref(lb.c), ctypes.byref(rb.c), ctypes.byref(Lo.c),
                                            ctypes.byref(Mo.c), ctypes.byref(Ro.c), ctypes.byref(w1.c),
                                            ctypes.byref(w2.c), ctypes.byref(opts), ctypes.byref(h)),
              "heff_vjp_plan_create")
        super().__init__(h, (lb, rb, Lo, Mo, Ro, w1, w2))
        self.lbond, self.rbond = lb, rb
        self.nnz1, self.nnz2 = len(w1.rows), len(w2.rows)

    def prepare(self, L, R):
        self._check_env(L, R)
        self._uploaded("heff_prepare")
        check(lib().hx_heff_prepare(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _stream()), "heff_prepare")
        self._ready = True

    def _check_backward(self, psi, g, g_psi, g_L, g_R, g_W1, g_W2, dtype, env=()):
        n = int(self.info.psi_nnz)
        need_all(self.device, *env, (psi, "psi", n, dtype), (g, "g", n, dtype), (g_psi, "g_psi", n, dtype),
                 (g_L, "g_L", int(self.info.in_nnz), dtype), (g_R, "g_R", int(self.info.in2_nnz), dtype),
                 (g_W1, "g_W1", 16 * self.nnz1, dtype), (g_W2, "g_W2", 16 * self.nnz2, dtype))
        if n and g_psi.data_ptr() in (psi.data_ptr(), g.data_ptr()):
            raise ValueError("g_psi must not alias psi or g")

    def backward(self, L, R, psi, g, g_psi, g_L, g_R, g_W1, g_W2):
        self._check_backward(psi, g, g_psi, g_L, g_R, g_W1, g_W2, "float64", env=self._env_items(L, R))
        self._prepared("heff_apply_backward")
        check(lib().hx_heff_apply_backward(self.h, _ptr(L), _ptr(R), _ptr(self.ws), _ptr(psi), _ptr(g), _ptr(g_psi),
                                           _ptr(g_L), _ptr(g_R), _ptr(g_W1), _ptr(g_W2), _stream()),
              "heff_apply_backward")

    def lower_f32(self, L, R):
        """FP32 copies of L, R, the prepared mixed operators and the coefficient table."""
        HeffPlan.lower_f32(self, L, R)

    def backward_f32(self, psi32, g32, g_psi32, g_L32, g_R32, g_W1_32, g_W2_32):
        self._check_backward(psi32, g32, g_psi32, g_L32, g_R32, g_W1_32, g_W2_32, "float32")
        self._lowered("heff_apply_backward_f32")
        check(lib().hx_heff_apply_backward_f32(self.h, _ptr(self.L32), _ptr(self.R32), _ptr(self.ws32), _ptr(psi32),
                                               _ptr(g32), _ptr(g_psi32), _ptr(g_L32), _ptr(g_R32), _ptr(g_W1_32),
                                               _ptr(g_W2_32), _stream()), "heff_apply_backward_f32")


class Heff1VjpPlan(HeffVjpPlan):
    """Plan of the vector-Jacobian products of the one-site sigma = H1 psi (psi in the
    one-site layout); nnz2 counts the identity coupling of the absent site."""

    def __init__(self, lbond, rbond, Ldq, Rdq, W, t_budget_bytes=0, split_kseg_min=0, kernel_variant=0):
        lb, rb = (b if isinstance(b, Bond) else Bond(b) for b in (lbond, rbond))
        Lo, Ro = OpSet(Ldq), OpSet(Rdq)
        w = W if isinstance(W, MpoSite) else MpoSite.from_entries(W)
        opts = _opts(t_budget_bytes, split_kseg_min, kernel_variant)
        h = c_void_p()
        check(lib().hx_heff1_vjp_plan_create(ctypes.byref(lb.c), ctypes.byref(rb.c), ctypes.byref(Lo.c),
                                             ctypes.byref(Ro.c), ctypes.byref(w.c), ctypes.byref(opts),
                                             ctypes.byref(h)), "heff1_vjp_plan_create")
        Plan.__init__(self, h, (lb, rb, Lo, Ro, w))
        self.lbond, self.rbond = lb, rb
        self.nnz1, self.nnz2 = len(w.rows), Ro.nop


GRAPH_APPLY, GRAPH_PREPARE_APPLY, GRAPH_APPLY_F32, GRAPH_APPLY_BF16 = 1, 2, 3, 4


class Graph:
    """An executable HIP graph of a plan's launch sequence with fixed operand
    tensors (kept alive here)."""

    def __init__(self, plan, what, L, R, ws, psi, sigma):
        h = c_void_p()
        check(lib().hx_heff_graph_create(plan.h, int(what), _ptr(L), _ptr(R), _ptr(ws), _ptr(psi), _ptr(sigma),
                                         ctypes.byref(h)), "heff_graph_create")
        self.h = h
        self._keep = (plan, L, R, ws, psi, sigma)

    def launch(self):
        check(lib().hx_graph_launch(self.h, _stream()), "graph_launch")

    def __del__(self):
        try:
            if self.h:
                lib().hx_graph_destroy(self.h)
                self.h = None
        except Exception:
            pass


class BatchPlan(HeffPlan):
    """Several sigma-vector plans merged into one launch sequence.  Operands of
    instance i live at `offsets[i] = (psi_off, L_off, R_off)` of the concatenated
    buffers."""

    def __init__(self, plans):
        arr = (c_void_p * len(plans))(*[p.h for p in plans])
        h = c_void_p()
        check(lib().hx_heff_plan_batch(arr, len(plans), ctypes.byref(h)), "heff_plan_batch")
        Plan.__init__(self, h, tuple(plans))
        self.offsets = []
        for i in range(len(plans)):
            o = [c_int64(), c_int64(), c_int64()]
            check(lib().hx_batch_offsets(self.h, i, *[ctypes.byref(x) for x in o]), "batch_offsets")
            self.offsets.append(tuple(int(x.value) for x in o))
        self.sizes = [(int(p.info.psi_nnz), int(p.info.in_nnz), int(p.info.in2_nnz)) for p in plans]


class EnvPlan(Plan):
    def __init__(self, direction, bond_in, bond_out, dq_in, dq_out, W, t_budget_bytes=0, split_kseg_min=0,
                 kernel_variant=0, b_part=0, b_nparts=1):
        bi, bo = (b if isinstance(b, Bond) else Bond(b) for b in (bond_in, bond_out))
        oi, oo = OpSet(dq_in), OpSet(dq_out)
        w = W if isinstance(W, MpoSite) else MpoSite.from_entries(W)
        opts = _opts(t_budget_bytes, split_kseg_min, kernel_variant, 1, b_part, b_nparts)
        h = c_void_p()
        check(lib().hx_env_plan_create(int(direction), ctypes.byref(bi.c), ctypes.byref(bo.c), ctypes.byref(oi.c),
                                       ctypes.byref(oo.c), ctypes.byref(w.c), ctypes.byref(opts), ctypes.byref(h)),
              "env_plan_create")
        super().__init__(h, (bi, bo, oi, oo, w))

    def update(self, env_in, site, env_out):
        need_all(self.device, (env_in, "env_in", int(self.info.in_nnz), "float64"),
                 (site, "site", int(self.info.in2_nnz), "float64"),
                 (env_out, "env_out", int(self.info.out_nnz), "float64"))
        self._uploaded("env_update")
        check(lib().hx_env_update(self.h, _ptr(env_in), _ptr(site), _ptr(self.ws), _ptr(env_out), _stream()),
              "env_update")


def davidson_ws_bytes(n, kmax):
    return int(lib().hx_davidson_ws_bytes(int(n), int(kmax)))


def davidson_step(n, k, kmax, V, S, diag, guard, ws, x, hx, t, scal):
    """Tensors: V, S (kmax, n) row-major float64; diag, x, hx, t (n,); ws bytes; scal (>=3,)."""
    if not 1 <= k <= kmax <= 32:
        raise ValueError("davidson_step: need 1 <= k <= kmax <= 32")
    for m, name in ((V, "V"), (S, "S")):
        if m.dim() != 2 or m.shape[0] < k or m.shape[1] < n or m.stride(1) != 1:
            raise ValueError(f"davidson_step: {name} must be a row-major (>= k, >= n) matrix")
    need_all(diag.device, (diag, "diag", n, "float64"), (x, "x", n, "float64"), (hx, "hx", n, "float64"),
             (t, "t", n, "float64"), (scal, "scal", 3, "float64"), (V, "V", 0, "float64"), (S, "S", 0, "float64"),
             (ws, "ws", davidson_ws_bytes(n, kmax) // ws.element_size(), str(ws.dtype).split(".")[-1]))
    check(lib().hx_davidson_step(int(n), int(k), int(kmax), _ptr(V), V.stride(0), _ptr(S), S.stride(0), _ptr(diag),
                                 float(guard), _ptr(ws), _ptr(x), _ptr(hx), _ptr(t), _ptr(scal), _stream()),
          "davidson_step")


def davidson_restart2(x, hx, xp, hxp, v1, s1, ws, scal):
    check(lib().hx_davidson_restart2(int(x.numel()), _ptr(x), _ptr(hx), _ptr(xp), _ptr(hxp), _ptr(v1), _ptr(s1),
                                     _ptr(ws), _ptr(scal), _stream()), "davidson_restart2")


def dots(a, b, ws, out):
    """out[j] = a[j] . b for a (k, n) float64 rows."""
    k, n = a.shape
    check(lib().hx_dots(int(n), int(k), _ptr(a), a.stride(0), _ptr(b), _ptr(ws), _ptr(out), _stream()), "dots")


def normalize(x, ws, norm_out=None):
    """x <- x / ||x|| in place (library kernel)."""
    check(lib().hx_normalize(int(x.numel()), _ptr(x), _ptr(ws), _ptr(norm_out), _stream()), "normalize")


def convert_f64_f32(src, dst):
    check(lib().hx_convert_f64_f32(int(src.numel()), _ptr(src), _ptr(dst), _stream()), "convert_f64_f32")


def convert_f32_f64(src, dst):
    check(lib().hx_convert_f32_f64(int(src.numel()), _ptr(src), _ptr(dst), _stream()), "convert_f32_f64")


def gather_index(idx, src, dst):
    """dst[j] = src[idx[j]] (device int64 idx of dst's length)."""
    if str(idx.dtype) != "torch.int64":
        raise TypeError("gather_index: idx must be int64")
    check(lib().hx_gather_index(int(dst.numel()), _ptr(idx), int(src.numel()), _ptr(src), _ptr(dst), _stream()),
          "gather_index")


def scatter_index(idx, src, dst):
    """dst[idx[j]] = src[j] (device int64 idx of src's length)."""
    if str(idx.dtype) != "torch.int64":
        raise TypeError("scatter_index: idx must be int64")
    check(lib().hx_scatter_index(int(src.numel()), _ptr(idx), int(dst.numel()), _ptr(src), _ptr(dst), _stream()),
          "scatter_index")


def axpy(a, x, y):
    """y += a x on the device."""
    check(lib().hx_axpy(int(x.numel()), float(a), _ptr(x), _ptr(y), _stream()), "axpy")
