"""Autotuner for the block-GEMM plans.

The kernel shape choices of a sigma-vector plan (hx_plan_opts) are tuned by
measurement on the problem itself: the kernel variant (LDS buffering, 16- or
8-deep K stages, the tile shapes 64 x 64 / 128 x 32 / 32 x 128 and single-wave
32 x 32 tiles), the minimum split-K segment and the intermediate budget (how many
middle-bond operators share one T chunk).  The search is greedy coordinate descent from the defaults: each axis
in turn is swept with the others fixed, and the best value kept.  Every
candidate's sigma is checked against the default plan's result before its time
counts, so a tuned plan is never a wrong plan.  Results are cached in a JSON
file keyed by the problem's shape signature.
"""

import hashlib
import json
import os

import numpy as np

AXES = (
    ("kernel_variant", (0, 1, 2, 4, 5, 6)),
    ("split_kseg_min", (512, 1024, 2048, 4096)),
    ("t_budget_bytes", (1 << 29, 1 << 30, 1 << 31)),
)
DEFAULT = {"kernel_variant": 0, "split_kseg_min": 2048, "t_budget_bytes": 1 << 30}


def coordinate_search(timer, axes=AXES, start=None):
    """Greedy coordinate descent.  `timer(opts)` returns seconds (or None when
    the candidate is rejected).  Returns (best_opts, {key: seconds})."""
    best = dict(DEFAULT if start is None else start)
    seen = {}

    def t(opts):
        k = json.dumps(opts, sort_keys=True)
        if k not in seen:
            seen[k] = timer(dict(opts))
        return seen[k]

    best_t = t(best)
    if best_t is None:
        raise RuntimeError("autotune: the starting options were rejected")
    for name, values in axes:
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best)
            cand[name] = v
            tc = t(cand)
            if tc is not None and tc < best_t:
                best, best_t = cand, tc
    return best, seen


def signature(lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, extra=""):
    h = hashlib.sha1()
    for b in (lbond, rbond):
        h.update(repr([(tuple(q), int(m)) for q, m in (b.sectors if hasattr(b, "sectors") else b)]).encode())
    for d in (Ldq, mid_dq, Rdq):
        h.update(np.ascontiguousarray(np.asarray(d, dtype=np.int32)).tobytes())
    for w in (W1, W2):
        h.update(np.ascontiguousarray(w.rows).tobytes() + np.ascontiguousarray(w.cols).tobytes())
        h.update(np.ascontiguousarray(w.vals).tobytes())
    h.update(extra.encode())
    return h.hexdigest()


def tune(build, apply, axes=AXES, reps=3, rtol=1e-11, start=None):
    """Generic measurement loop: `build(opts)` returns an uploaded, prepared plan
    and `apply(plan)` runs its step and returns the output tensor.  Returns
    (best_opts, timings)."""
    import torch
    ref = {}

    def timer(opts):
        plan = build(opts)
        out = apply(plan)
        torch.cuda.synchronize()
        if "out" not in ref:
            ref["out"] = out.clone()
            ref["scale"] = float(out.abs().max())
        elif float((out - ref["out"]).abs().max()) > rtol * max(ref["scale"], 1e-300):
            return None
        ts = []
        for _ in range(reps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            apply(plan)
            e.record()
            e.synchronize()
            ts.append(s.elapsed_time(e) / 1e3)
        del plan
        return float(np.median(ts))

    return coordinate_search(timer, axes, start)


def tune_heff(lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, L, R, psi, reps=3, cache_path=None, axes=AXES,
              rtol=1e-11):
    """Tune the options of one FP64 sigma-vector plan on the GPU; returns
    (best_opts, timings).  L, R, psi: device tensors in the library layouts."""
    import torch
    from . import _lib as X
    W1 = W1 if isinstance(W1, X.MpoSite) else X.MpoSite.from_entries(W1)
    W2 = W2 if isinstance(W2, X.MpoSite) else X.MpoSite.from_entries(W2)
    key = signature(lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, torch.cuda.get_device_name())
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["timings"]
    sig = torch.empty_like(psi)

    def build(opts):
        plan = X.HeffPlan(lbond, rbond, Ldq, mid_dq, Rdq, W1, W2, **opts).upload(psi.device)
        plan.prepare(L, R)
        return plan

    def apply(plan):
        plan.apply(L, R, psi, sig)
        return sig

    best, timings = tune(build, apply, axes, reps, rtol)
    if cache_path:
        cache[key] = {"best": best, "timings": timings}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best, timings
