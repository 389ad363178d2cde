"""Benchmark: one two-site DMRG step at the middle of a 36-orbital ab initio chain.

Workload (synthetic; the paper's molecular integrals are not available): seeded
Gaussian integrals for 36 orbitals, 36 electrons, 2Sz = 0; bond dimension
M = 1000 with a Gaussian sector distribution; environments are the real
renormalised operators of a seeded random MPS, built on the GPU by environment
updates from both ends (untimed setup).

One timed step = the whole hot path at sites (17, 18): operator mixing, diag,
Davidson (sigma = H_eff psi + Davidson steps) to |r| <= 1e-7, SVD split of the
Ritz vector, environment update.  The Davidson start vector is warm, as in a
step after the first sweep: the Ritz vector of an untimed 100-iteration FP64
solve from a seeded random vector.  The FP64 reference energy comes from an
untimed FP64 solve to |r| <= 1e-9.  `value` is the algorithmic FLOP of the
step's GEMM work divided by its wall time.  --mode f32 runs the block
contractions in FP32 (FP32 MFMA accumulation) until |r| <= 1e-5, then refines
with FP64 sigma-vectors; the Davidson vector work is FP64 in both modes.

Prints one JSON line.  Only one GPU is supported.
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H_eff·ψ GFLOP/s & %MFMA peak at M=1000; Davidson energy err vs FP64 oracle"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAKS = {"f64": PEAK_FP64_TFLOPS, "f32": PEAK_FP32_TFLOPS, "bf16": PEAK_BF16_TFLOPS}
PEAK_HBM_GBS = 8000.0
# HBM bytes of one FP64 sigma-vector at the default workload (36 orbitals, M = 1000,
# middle step) from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by what the counters
# read for a device copy of known size), per plan options (kernel_variant,
# split_kseg_min, intermediate budget), with the summary they come from.  Only valid
# for the kernel and plan builder they were taken with; other options report null.
# (kernel_variant, split_kseg_min, intermediate budget, merged intermediates off)
MEASURED_TRAFFIC = {(1, 512, 1 << 30, 0): (86.22e9, "profiles/bsgemm_f64_apply_traffic_K36_M1000.md"),
                    (1, 512, 1 << 31, 0): (85.04e9, "profiles/bsgemm_f64_apply_traffic_K36_M1000.md"),
                    (1, 1024, 1 << 30, 0): (85.06e9, "profiles/bsgemm_f64_apply_traffic_K36_M1000.md"),
                    (1, 1024, 1 << 31, 0): (85.23e9, "profiles/bsgemm_f64_apply_traffic_K36_M1000.md")}
# The same for one batched sigma-vector of the default batch (16 instances, 16 orbitals,
# M = 256, every instance in one intermediate chunk), keyed by (kernel_variant,
# split_kseg_min, merged intermediates off).
MEASURED_BATCH_TRAFFIC = {(6, 512, 0): (14.67e9, "profiles/bsgemm_batch_16x_K16_M256.md")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_environments(X, mpo, bonds, left, right, i, device):
    """Left environment at cut i and right environment at cut i+2 via GPU updates."""
    import torch
    from paper_2310_03920_amd.engine import site_payload
    K = mpo.K
    W = [X.MpoSite(s.rows, s.cols, s.mats) for s in mpo.sites]

    def lplan(k):
        return X.EnvPlan(0, bonds[k], bonds[k + 1], mpo.dq[k], mpo.dq[k + 1], W[k])

    def rplan(k):
        return X.EnvPlan(1, bonds[k + 1], bonds[k], mpo.dq[k + 1], mpo.dq[k], W[k])

    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        lp = list(ex.map(lplan, range(i)))
        rp = list(ex.map(rplan, range(K - 1, i + 1, -1)))
    log(f"env plans built in {time.time() - t0:.1f}s")
    Lenv = torch.ones(1, dtype=torch.float64, device=device)
    for k, p in zip(range(i), lp):
        p.upload(device)
        out = torch.empty(int(p.info.out_nnz), dtype=torch.float64, device=device)
        p.update(Lenv, site_payload(bonds[k], bonds[k + 1], left[k], device), out)
        Lenv = out
        p.tables = p.ws = None
    Renv = torch.ones(1, dtype=torch.float64, device=device)
    for k, p in zip(range(K - 1, i + 1, -1), rp):
        p.upload(device)
        out = torch.empty(int(p.info.out_nnz), dtype=torch.float64, device=device)
        p.update(Renv, site_payload(bonds[k], bonds[k + 1], right[k], device), out)
        Renv = out
        p.tables = p.ws = None
    torch.cuda.synchronize()
    log(f"environments built in {time.time() - t0:.1f}s")
    return Lenv, Renv


def cpu_baseline(mpo, bonds, i, stride=8, seed=5):
    """Time the FP64 block-sparse oracle sigma (oracle.blocks: one numpy matmul per
    block product, iterating over output column blocks) on the host, on the same
    shapes and MPO with seeded random environments and psi.  The sample is the sum
    over every `stride`-th middle-bond index b (the terms of different b are
    independent); its FLOP count is the oracle's own count of block-product work.
    Timed with the BLAS pool at all host threads and at one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import blocks
    from paper_2310_03920_amd.mpo import site_entries
    from synth.blocks import random_env, random_psi
    rng = np.random.default_rng(seed)
    lb, rb = bonds[i], bonds[i + 2]
    L = random_env(lb, [tuple(x) for x in mpo.dq[i]], rng)
    R = random_env(rb, [tuple(x) for x in mpo.dq[i + 2]], rng)
    psi = random_psi(lb, rb, rng)
    W1, W2 = site_entries(mpo, i), site_entries(mpo, i + 1)
    nmid = len(mpo.dq[i + 1])
    bsel = list(range(0, nmid, stride))
    mixed = blocks.prepare(L, W1, W2, R, bsel)
    ncpu = os.cpu_count() or 1
    legs = {}
    for nt in (ncpu, 1):
        with threadpool_limits(limits=nt):
            used = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] + [1])
            fl = [0.0]
            t0 = time.time()
            blocks.heff_apply(lb, rb, L, W1, W2, R, psi, bsel=bsel, flops=fl, mixed=mixed)
            dt = time.time() - t0
        legs[nt] = (fl[0] / dt / 1e9, used, dt, fl[0])
    rate, used, dt, fl = legs[ncpu]
    return {"value": rate, "unit": "GFLOP/s", "cores": int(used), "kind": "oracle",
            "sample": f"oracle.blocks sigma (FP64 numpy, one matmul per block product) restricted to "
                      f"{len(bsel)} of {nmid} middle-bond indices (every {stride}th b): {fl / 1e9:.1f} GFLOP "
                      f"of block products in {dt:.1f}s",
            "value_1thread": legs[1][0], "seconds_1thread": legs[1][2], "host_cpus": ncpu}


def calibration_copy(device):
    """A plain device copy of known size (2^26 doubles read, 2^26 written) that closes
    a run: per-dispatch HBM byte counters of the run's kernels are scaled by what the
    same counters read for it."""
    import torch
    src = torch.ones(1 << 26, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def batch_instances(X, M=256, K=16, count=16):
    """The mixed-size batch: `count` independent two-site problems of a K-orbital
    chain at bond dimension M; instance j (1-based) has integrals seed j,
    N = 14/16/18 electrons (j mod 3) and centre sites (i, i+1), i = 2 + 5j mod 12."""
    from paper_2310_03920_amd.mpo import build_nc_mpo
    from synth import bond_sector_tables, make_integrals
    out = []
    for j in range(1, count + 1):
        N = (14, 16, 18)[j % 3]
        i = 2 + (5 * j) % 12
        mpo = build_nc_mpo(*make_integrals(K, seed=j))
        bonds = bond_sector_tables(K, N, 0, M, model="gaussian", width=1.0)
        out.append(dict(j=j, N=N, i=i, mpo=mpo, lbond=bonds[i], rbond=bonds[i + 2],
                        W1=X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats),
                        W2=X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats)))
    return out


def bench_batch(args):
    """Throughput of many small sigma-vectors: one by one (eager) vs one batched
    plan (eager and replayed from a HIP graph)."""
    import torch
    from paper_2310_03920_amd import _lib as X
    X.lib()
    device = "cuda"
    t0 = time.time()
    insts = batch_instances(X, M=args.bond_dim, K=args.orbitals, count=args.instances)

    # intermediate budget per instance: by default every instance in one chunk
    budget = int(args.batch_t_budget_mb * (1 << 20)) if args.batch_t_budget_mb else 1 << 40

    def make_plans(opts):
        ps = []
        for d in insts:
            m = d["mpo"]
            i = d["i"]
            ps.append(X.HeffPlan(d["lbond"], d["rbond"], m.dq[i], m.dq[i + 1], m.dq[i + 2], d["W1"], d["W2"],
                                 t_budget_bytes=budget, **opts))
        return ps

    opts = {"split_kseg_min": args.kseg or 2048, "kernel_variant": 0 if args.variant is None else args.variant,
            "t_merge_off": int(args.no_t_merge)}
    plans = make_plans(opts)
    log(f"{len(plans)} plans in {time.time() - t0:.1f}s")
    gen = torch.Generator(device=device)
    gen.manual_seed(11)

    def rnd(n):
        return torch.randn(max(int(n), 1), generator=gen, dtype=torch.float64, device=device)

    Ls = [rnd(p.info.in_nnz) for p in plans]
    Rs = [rnd(p.info.in2_nnz) for p in plans]
    Ps = [rnd(p.info.psi_nnz) for p in plans]
    Ss = [torch.empty_like(x) for x in Ps]
    Lc = torch.cat([x[:int(p.info.in_nnz)] for x, p in zip(Ls, plans)])
    Rc = torch.cat([x[:int(p.info.in2_nnz)] for x, p in zip(Rs, plans)])
    Pc = torch.cat([x[:int(p.info.psi_nnz)] for x, p in zip(Ps, plans)])
    Sc = torch.empty_like(Pc)
    tune_s = 0.0
    if not args.no_autotune:
        from paper_2310_03920_amd import autotune
        axes = [a for a in autotune.AXES[:2] if not (a[0] == "kernel_variant" and args.variant is not None)
                and not (a[0] == "split_kseg_min" and args.kseg)]

        if args.mode == "bf16":  # BF16 products need 16-deep stages and 4-wave tiles
            axes = [(k, tuple(v for v in vals if v not in (2, 6))) if k == "kernel_variant" else (k, vals)
                    for k, vals in axes]
        Pt32, St32 = Pc.float(), torch.empty_like(Pc, dtype=torch.float32)

        def build(o):
            b = X.BatchPlan(make_plans(o)).upload(device)
            b.prepare(Lc, Rc)
            if args.mode != "f64":
                b.lower_f32(Lc, Rc)
            return b

        def run(b):
            # tuned on the sigma-vector of the benchmarked precision
            if args.mode == "f64":
                b.apply(Lc, Rc, Pc, Sc)
                return Sc
            (b.apply_bf16 if args.mode == "bf16" else b.apply_f32)(Pt32, St32)
            return St32

        t1 = time.time()
        opts, timings = autotune.tune(build, run, axes=axes, reps=3, start=opts,
                                      rtol={"f64": 1e-11, "f32": 1e-4, "bf16": 1e-2}[args.mode])
        tune_s = time.time() - t1
        log(f"autotune in {tune_s:.1f}s: {opts} "
            f"({', '.join(f'{k}: {1e3 * v:.2f} ms' for k, v in timings.items() if v is not None)})")
        plans = make_plans(opts)
    B = X.BatchPlan(plans).upload(device)
    for p in plans:
        p.upload(device)
    log(f"batch {B.info.flops_apply / 1e9:.2f} GFLOP/apply, tiles {B.info.n_tiles}, ws {B.info.ws_bytes / 1e9:.2f} GB")
    f32 = args.mode != "f64"
    bf = args.mode == "bf16"
    for p, L, R in zip(plans, Ls, Rs):
        p.prepare(L, R)
        if f32:
            p.lower_f32(L, R)
    B.prepare(Lc, Rc)
    if f32:
        B.lower_f32(Lc, Rc)
        P32 = [x.float() for x in Ps]
        S32 = [torch.empty_like(x) for x in P32]
        Pc32, Sc32 = Pc.float(), torch.empty_like(Pc, dtype=torch.float32)
        graph = X.Graph(B, X.GRAPH_APPLY_BF16 if bf else X.GRAPH_APPLY_F32, B.L32, B.R32, B.ws32, Pc32, Sc32)

        def one_by_one():
            for p, x, y in zip(plans, P32, S32):
                (p.apply_bf16 if bf else p.apply_f32)(x, y)

        def batched():
            (B.apply_bf16 if bf else B.apply_f32)(Pc32, Sc32)
    else:
        graph = X.Graph(B, X.GRAPH_APPLY, Lc, Rc, B.ws, Pc, Sc)

        def one_by_one():
            for p, L, R, x, y in zip(plans, Ls, Rs, Ps, Ss):
                p.apply(L, R, x, y)

        def batched():
            B.apply(Lc, Rc, Pc, Sc)

    # batched output == instance outputs, bit for bit
    one_by_one()
    batched()
    torch.cuda.synchronize()
    outs = S32 if f32 else Ss
    bout = Sc32 if f32 else Sc
    for (po, _, _), y in zip(B.offsets, outs):
        n = y.numel() if not f32 else y.numel()
        if not torch.equal(bout[po:po + n], y[:n]):
            raise RuntimeError("batched sigma differs from the instance sigma")

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = time.perf_counter()
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps / 1e3, (time.perf_counter() - ts) / reps

    reps = max(args.steps, 1) * 10
    t_one, w_one = timed(one_by_one, reps)
    t_bat, w_bat = timed(batched, reps)
    t_gr, w_gr = timed(graph.launch, reps)
    calibration_copy(device)
    fl = B.info.flops_useful
    peak = PEAKS[args.mode]
    achieved = fl / t_gr / 1e12
    gbs = B.info.bytes_apply / t_gr / 1e9
    default_batch = (args.instances, args.orbitals, args.bond_dim, budget) == (16, 16, 256, 1 << 40)
    traffic = (MEASURED_BATCH_TRAFFIC.get((opts["kernel_variant"], opts["split_kseg_min"], opts.get("t_merge_off", 0)))
               if args.mode == "f64" and default_batch else None)
    out = {
        "metric": METRIC,
        "value": fl / w_gr / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * w_gr,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.mode,
        "data": "synthetic",
        "config": {
            "workload": f"batch of {len(plans)} independent two-site sigma-vectors, {args.orbitals}-orbital ab initio "
                        f"chains, M={args.bond_dim} (Gaussian sectors), N in 14/16/18, centres 2..13, "
                        f"integral seeds 1..{len(plans)}, random N(0,1) environments; one step = one batched "
                        f"sigma-vector replayed from a HIP graph",
            "instances": len(plans), "bond_dim": args.bond_dim, "orbitals": args.orbitals,
            "psi_nnz_total": int(B.info.psi_nnz), "tiles": int(B.info.n_tiles), "plan_opts": opts,
            "t_budget_per_instance_bytes": budget, "rounds_chunks": int(B.info.n_chunks),
            "autotune_s": tune_s,
        },
        "batch": {"gflop": fl / 1e9, "one_by_one_ms": 1e3 * t_one, "batched_ms": 1e3 * t_bat,
                  "graph_ms": 1e3 * t_gr, "one_by_one_wall_ms": 1e3 * w_one, "batched_wall_ms": 1e3 * w_bat,
                  "graph_wall_ms": 1e3 * w_gr, "speedup_vs_one_by_one": t_one / t_gr},
        # the batch's arithmetic intensity is below the FP64 ridge: its roof is HBM bandwidth
        # over its algorithmic bytes (each operand block, psi, sigma and the intermediates once)
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": traffic[0] if traffic else None,
                     "traffic_source": traffic[1] if traffic else None,
                     "traffic_unit": "HBM bytes per batched sigma-vector (rocprofv3 FETCH_SIZE + WRITE_SIZE, stored)",
                     "bytes_algorithmic": float(B.info.bytes_apply),
                     "flops": {"achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak},
                     "kernel": "bsgemm (every launch of one batched sigma-vector, graph replay)"},
    }
    print(json.dumps(out), flush=True)


def plan_options(args, X, mpo, bonds, i, Lenv, Renv, tb, device):
    """Plan options of the middle step: tuned on the GPU (untimed setup) unless
    --no-autotune; explicit --variant / --kseg pin those axes."""
    import torch
    from paper_2310_03920_amd import autotune
    from synth.blocks import random_psi
    opts = {"t_budget_bytes": tb, "split_kseg_min": args.kseg or 2048,
            "kernel_variant": 0 if args.variant is None else args.variant,
            "t_merge_off": int(args.no_t_merge)}
    if args.no_autotune:
        return opts, 0.0
    axes = [a for a in autotune.AXES if not (a[0] == "kernel_variant" and args.variant is not None)
            and not (a[0] == "split_kseg_min" and args.kseg)]
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    psi = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], np.random.default_rng(9)))).to(device)
    W1 = X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats)
    W2 = X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats)
    sig = torch.empty_like(psi)
    psi32, sig32 = psi.float(), torch.empty_like(psi, dtype=torch.float32)
    if args.mode == "bf16":  # BF16 products need 16-deep stages and 4-wave tiles
        axes = [(k, tuple(v for v in vals if v not in (2, 6))) if k == "kernel_variant" else (k, vals) for k, vals in axes]

    def build(o):
        p = X.HeffPlan(lb, rb, mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2], W1, W2, **o).upload(device)
        p.prepare(Lenv, Renv)
        if args.mode != "f64":
            p.lower_f32(Lenv, Renv)
        return p

    def run(p):
        # tuned on the sigma-vector of the benchmarked precision
        if args.mode == "f64":
            p.apply(Lenv, Renv, psi, sig)
            return sig
        (p.apply_bf16 if args.mode == "bf16" else p.apply_f32)(psi32, sig32)
        return sig32

    t0 = time.time()
    best, timings = autotune.tune(build, run, axes=axes, reps=2, start=opts,
                                  rtol={"f64": 1e-11, "f32": 1e-4, "bf16": 1e-2}[args.mode])
    log(f"autotune in {time.time() - t0:.1f}s: {best} "
        f"({', '.join(f'{k}: {1e3 * v:.1f} ms' for k, v in timings.items() if v is not None)})")
    torch.cuda.empty_cache()
    return best, time.time() - t0


def apply_only(args, X, mpo, bonds, i, Lenv, Renv, opts, tune_s, device):
    """Time bare sigma-vectors (FP64, or FP32 with --mode f32) at the middle step."""
    import torch
    from synth.blocks import random_psi
    plan = X.HeffPlan(bonds[i], bonds[i + 2], mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2],
                      X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats),
                      X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats),
                      n_roots=args.roots, **opts).upload(device)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    rng = np.random.default_rng(3)
    psis = [X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], rng)) for _ in range(args.roots)]
    psi = torch.from_numpy(X.pack_roots(lb, rb, psis) if args.roots > 1 else psis[0]).to(device)
    sig = torch.empty_like(psi)
    plan.prepare(Lenv, Renv)
    f32 = args.mode != "f64"
    if f32:
        plan.lower_f32(Lenv, Renv)
        psi32, sig32 = psi.float(), torch.empty_like(psi, dtype=torch.float32)
        low = plan.apply_bf16 if args.mode == "bf16" else plan.apply_f32

    def one():
        if f32:
            low(psi32, sig32)
        else:
            plan.apply(Lenv, Renv, psi, sig)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    ms = []
    for _ in range(args.steps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        one()
        e.record()
        e.synchronize()
        ms.append(s.elapsed_time(e))
    info = plan.info
    avg = float(np.mean(ms)) / 1e3
    peak = PEAKS[args.mode]
    achieved = info.flops_useful / avg / 1e12
    parts = middle_bond_parts(args, X, mpo, bonds, i, Lenv, Renv, opts, psi, device) if args.bparts > 1 else None
    # counter traffic stored for this plan (FP64, the default 36-orbital M = 1000 workload)
    traffic = (MEASURED_TRAFFIC.get((opts["kernel_variant"], opts["split_kseg_min"], opts["t_budget_bytes"],
                                     opts.get("t_merge_off", 0)))
               if args.mode == "f64" and (mpo.K, args.bond_dim) == (36, 1000) and args.partition == "nc" else None)
    calibration_copy(device)
    print(json.dumps({
        "metric": METRIC, "value": info.flops_useful / avg / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * avg, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.mode, "data": "synthetic",
        "config": {"workload": f"sigma-vectors only at sites ({i},{i + 1}) of the {mpo.K}-orbital chain, "
                               f"M={args.bond_dim}, {args.roots} vector(s) per call, "
                               + ("NC-partition MPO" if args.partition == "nc" else f"NC->CN switch at cut {mpo.K // 2}"),
                   "roots": args.roots, "tflop_per_call": info.flops_useful / 1e12,
                   "tflop_executed_per_call": info.flops_apply / 1e12,
                   "mpo_bond_dims": [len(mpo.cuts[k]) for k in (i, i + 1, i + 2)],
                   "chunks": int(info.n_chunks), "tiles": int(info.n_tiles),
                   "apply_ms_each": ms, "plan_opts": opts, "autotune_s": tune_s},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic[0] if traffic else None,
                     "traffic_source": traffic[1] if traffic else None},
        **({"middle_bond_parts": parts} if parts else {}),
    }), flush=True)


def middle_bond_parts(args, X, mpo, bonds, i, Lenv, Renv, opts, psi, device):
    """One GPU's share of the sigma-vector sharded over the MPO middle-bond index
    (Sec. II.B.1): plans restricted to b = p (mod n) for p = 0..n-1, each timed
    alone at the full operand shape, and the sum of the partial sigmas checked
    against the whole.  FP64 only."""
    import torch
    if args.mode != "f64":
        raise SystemExit("--bparts times the FP64 sigma-vector only")
    W1 = X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats)
    W2 = X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats)
    whole = torch.empty_like(psi)
    ref = X.HeffPlan(bonds[i], bonds[i + 2], mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2], W1, W2,
                     n_roots=args.roots, **opts).upload(device)
    ref.prepare(Lenv, Renv)
    ref.apply(Lenv, Renv, psi, whole)
    del ref
    total = torch.zeros_like(psi)
    part = torch.empty_like(psi)
    rows = []
    for p in range(args.bparts):
        plan = X.HeffPlan(bonds[i], bonds[i + 2], mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2], W1, W2,
                          n_roots=args.roots, b_part=p, b_nparts=args.bparts, **opts).upload(device)
        plan.prepare(Lenv, Renv)
        for _ in range(max(args.warmup, 1)):
            plan.apply(Lenv, Renv, psi, part)
        torch.cuda.synchronize()
        total += part
        ms = []
        for _ in range(args.steps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            plan.apply(Lenv, Renv, psi, part)
            e.record()
            e.synchronize()
            ms.append(s.elapsed_time(e))
        t = float(np.mean(ms))
        rows.append({"part": p, "ms": t, "tflop": plan.info.flops_useful / 1e12,
                     "tflops_per_s": plan.info.flops_useful / t / 1e9})
        log(f"middle-bond part {p}/{args.bparts}: {t:.2f} ms, {plan.info.flops_useful / 1e12:.3f} TFLOP")
        del plan
        torch.cuda.empty_cache()
    err = float((total - whole).abs().max()) / float(whole.abs().max())
    worst = max(r["ms"] for r in rows)
    return {"n_parts": args.bparts, "rule": "b mod n_parts", "parts": rows, "max_part_ms": worst,
            "sum_part_ms": sum(r["ms"] for r in rows),
            "flop_imbalance": max(r["tflop"] for r in rows) / (sum(r["tflop"] for r in rows) / len(rows)),
            "time_imbalance": worst / (sum(r["ms"] for r in rows) / len(rows)),
            "sum_of_parts_rel_err": err}


def bench_sweep(args):
    """Whole two-site passes (Sec. II.A.2) of the 24-orbital chain at M=500 from a
    seeded random MPS: every site step runs plan, prepare, diag, Davidson on the
    GPU sigma-vector, the host split and the GPU environment update.  One "step"
    of this workload is one pass (alternating directions, the first left to right)."""
    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.dmrg import DMRG
    from synth import make_integrals
    X.lib()
    K, M = args.orbitals, args.bond_dim
    h, g = make_integrals(K, seed=0)
    t0 = time.time()
    switch = K // 2 if args.partition == "nc-cn" else None
    d = DMRG(h, g, K, 0, M, seed=0, device="cuda", tol=args.tol, max_iter=args.max_iter, mpo_switch=switch,
             precision=args.mode, kmax=args.kmax)
    torch.cuda.synchronize()
    log(f"set-up (MPO, random MPS, right environments) {time.time() - t0:.1f}s; "
        f"MPO bond dims {[len(x) for x in d.mpo.dq]}")
    passes = []
    for p in range(args.steps):
        n0 = len(d.log)
        torch.cuda.synchronize()
        t = time.perf_counter()
        if p % 2 == 0:
            d.sweep_left_to_right(p, 0 if p == 0 else 1)
        else:
            d.sweep_right_to_left(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = d.log[n0:]
        passes.append({"s": dt, "site_steps": len(st), "matvecs": int(sum(x["n_matvec"] for x in st)),
                       "sigma_tflop": sum(x["n_matvec"] * x["sigma_flop"] for x in st) / 1e12,
                       "host_wall_s": {k: sum(x.get(k, 0.0) for x in st)
                                       for k in ("t_contract", "t_plan", "t_solve", "t_split", "t_env")},
                       "energy_last": st[-1]["energy"], "energy_min": min(x["energy"] for x in st)})
        log(f"pass {p}: {dt:.2f}s, {len(st)} site steps, {passes[-1]['matvecs']} sigma-vectors, "
            f"E = {st[-1]['energy']:.10f}")
    avg = sum(x["s"] for x in passes) / len(passes)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's block-sparse sigma at the middle site pair of the final MPS
        # bonds, on every 4th middle-bond index, scaled to the sigma work of an
        # average pass (sigma-vectors only: the host Davidson, split and
        # environment updates of a CPU sweep would come on top)
        i_mid = K // 2 - 1
        cb = cpu_baseline(d.mpo, d.bonds, i_mid, stride=4)
        work = sum(x["sigma_tflop"] for x in passes) / len(passes) * 1e12
        cpu = {"value": work / (cb["value"] * 1e9), "unit": "s/pass", "cores": cb["cores"], "kind": "oracle",
               "sample": cb["sample"] + f" at sites ({i_mid},{i_mid + 1}); {cb['value']:.1f} GFLOP/s applied to the "
                         f"{work / 1e12:.2f} TFLOP of sigma-vector work of an average pass (sigma-vectors only)",
               "value_1thread": work / (cb["value_1thread"] * 1e9), "oracle_gflops": cb["value"],
               "oracle_gflops_1thread": cb["value_1thread"], "host_cpus": cb["host_cpus"]}
        log(f"cpu baseline: {cpu['value']:.1f} s/pass at {cb['value']:.1f} GFLOP/s ({cb['cores']} threads)")
    print(json.dumps({
        "metric": "two-site DMRG pass wall time", "value": avg, "unit": "s/pass", "n_gpus": 1,
        "steps": args.steps, "warmup": 0, "ms_per_step": 1e3 * avg, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": args.mode, "data": "synthetic",
        "config": {"workload": f"two-site DMRG passes over a {K}-orbital ab initio chain, {K} electrons, "
                               f"2Sz=0, M={M}, integrals seed 0, seeded random initial MPS, "
                               + ("NC-partition MPO" if switch is None else f"NC-partition MPO up to cut {switch}, CN after"),
                   "orbitals": K, "bond_dim": M, "davidson": {"tol": args.tol, "max_iter": args.max_iter},
                   "mpo_bond_dims": [len(x) for x in d.mpo.dq]},
        "passes": passes, "peak_gpu_gb": torch.cuda.max_memory_allocated() / 1e9, "cpu_baseline": cpu}))


def mixed_compare(args, X, mpo, bonds, i, Lenv, Renv, opts, tune_s, device, seeds=5):
    """Mixed-precision Davidson against plain FP64 at equal accuracy, at the middle
    step: from `seeds` warm starts (each the Ritz vector of an untimed FP64 pre-solve
    from its own seeded random vector), solve to |r| <= tol with FP64 sigma-vectors,
    and with FP32 / BF16 sigma-vectors followed by FP64 refinement; time each solve
    (sigma-vectors and Davidson steps) and compare its energy with a tight FP64
    reference.  Prints one JSON line; `value` is FP64 time / best mixed time."""
    import torch
    from paper_2310_03920_amd.dmrg import PRECISIONS, Davidson
    from synth.blocks import random_psi
    plan = X.HeffPlan(bonds[i], bonds[i + 2], mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2],
                      X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats),
                      X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats),
                      **opts).upload(device)
    info = plan.info
    n = int(info.psi_nnz)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    diag = torch.empty(n, dtype=torch.float64, device=device)
    plan.prepare(Lenv, Renv)
    plan.diag(Lenv, Renv, diag)
    plan.lower_f32(Lenv, Renv)
    dav = Davidson(n, args.kmax, device)
    v32 = torch.empty(n, dtype=torch.float32, device=device)
    s32 = torch.empty(n, dtype=torch.float32, device=device)

    def mv(v, out):
        plan.apply(Lenv, Renv, v, out)

    def low(mode):
        ap = plan.apply_bf16 if mode == "bf16" else plan.apply_f32

        def mv_low(v, out):
            X.convert_f64_f32(v, v32)
            ap(v32, s32)
            X.convert_f32_f64(s32, out)
        return mv_low

    # per-sigma times of each precision (HIP events around 10 applies each)
    psi_t = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], np.random.default_rng(1)))).to(device)
    out_t = torch.empty_like(psi_t)
    sig_ms = {}
    for mode, fn in (("f64", mv), ("f32", low("f32")), ("bf16", low("bf16"))):
        fn(psi_t, out_t)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(10):
            fn(psi_t, out_t)
        e.record()
        e.synchronize()
        sig_ms[mode] = s.elapsed_time(e) / 10
    log(f"sigma-vector ms: {sig_ms}")
    starts = []
    for sd in range(seeds):
        p0 = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2],
                                                           np.random.default_rng(100 + sd)))).to(device)
        _, r_pre, _ = dav.solve(mv, p0, diag, tol=1e-12, max_iter=args.pre_iter)
        starts.append((dav.x.clone(), r_pre))
    e_ref, r_ref, n_ref = dav.solve(mv, starts[0][0], diag, tol=1e-10, max_iter=800)
    log(f"reference E = {e_ref:.12f} (|r| {r_ref:.1e}, {n_ref} sigma-vectors); warm starts |r| = "
        f"{[round(r, 5) for _, r in starts]}")
    runs = {"f64": [], "f32": [], "bf16": []}
    for sd, (x0, r_pre) in enumerate(starts):
        for mode in ("f64", "f32", "bf16"):
            torch.cuda.synchronize()
            t = time.perf_counter()
            if mode == "f64":
                th, rn, nh = dav.solve(mv, x0, diag, tol=args.tol, max_iter=args.max_iter)
                nl = 0
            else:
                th, rn, nl, nh = dav.solve_mixed(low(mode), mv, x0, diag, tol=args.tol, max_iter=args.max_iter,
                                                 **PRECISIONS[mode])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            runs[mode].append({"seed": sd, "s": dt, "energy_err": abs(th - e_ref), "rnorm": rn, "low_sigma": nl,
                               "f64_sigma": nh, "f64_equivalent_sigma": nh + nl * sig_ms[mode] / sig_ms["f64"]})
            log(f"seed {sd} {mode}: {dt:.2f}s, |dE| {abs(th - e_ref):.1e}, |r| {rn:.1e}, sigma {nl} low + {nh} f64")
    summ = {}
    for mode, rs in runs.items():
        ts = [r["s"] for r in rs]
        summ[mode] = {"mean_s": float(np.mean(ts)), "min_s": float(np.min(ts)), "max_s": float(np.max(ts)),
                      "mean_f64_equivalent_sigma": float(np.mean([r["f64_equivalent_sigma"] for r in rs])),
                      "max_energy_err": float(max(r["energy_err"] for r in rs)),
                      "max_rnorm": float(max(r["rnorm"] for r in rs))}
    f64_mean = summ["f64"]["mean_s"]
    spread = (summ["f64"]["max_s"] - summ["f64"]["min_s"]) / f64_mean
    best = min(("f32", "bf16"), key=lambda m: summ[m]["mean_s"])
    for mode in ("f32", "bf16"):
        summ[mode]["speedup_vs_f64"] = f64_mean / summ[mode]["mean_s"]
        summ[mode]["win_exceeds_f64_spread"] = bool(summ[mode]["mean_s"] < summ["f64"]["min_s"])
    print(json.dumps({
        "metric": "mixed-precision Davidson solve time vs FP64 at equal accuracy (middle step)",
        "value": f64_mean / summ[best]["mean_s"], "unit": "x (FP64 time / best mixed time)", "n_gpus": 1,
        "steps": seeds, "warmup": 0, "ms_per_step": 1e3 * summ[best]["mean_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": best, "data": "synthetic",
        "config": {"workload": f"Davidson solves at sites ({i},{i + 1}) of the {mpo.K}-orbital chain, M={args.bond_dim}, "
                               f"{seeds} seeded warm starts ({args.pre_iter} untimed FP64 iterations each), "
                               f"to |r| <= {args.tol}",
                   "sigma_ms": sig_ms, "reference_energy": e_ref, "reference_rnorm": r_ref,
                   "f64_time_spread": spread, "plan_opts": opts, "autotune_s": tune_s,
                   "precisions": {k: v for k, v in PRECISIONS.items()}},
        "summary": summ, "runs": runs}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--orbitals", type=int, default=36)
    ap.add_argument("--bond-dim", type=int, default=1000)
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--kmax", type=int, default=24, help="Davidson subspace size (at most 32)")
    ap.add_argument("--pre-iter", type=int, default=100)
    ap.add_argument("--t-budget-gb", type=float, default=1.0)
    ap.add_argument("--batch-t-budget-mb", type=float, default=0.0,
                    help="batch: intermediate budget per instance in MiB (0: one chunk per instance)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["f64", "f32", "bf16"], default="f64",
                    help="precision of the block contractions; Davidson is FP64 in all")
    ap.add_argument("--workload", choices=["middle", "batch", "apply", "sweep", "mixed"], default="middle",
                    help="middle: one DMRG step at the chain's middle; batch: many small sigma-vectors; "
                         "apply: sigma-vectors only at the middle step (profiling), ending with a 512 MiB "
                         "device copy that calibrates HBM byte counters; sweep: whole two-site passes "
                         "(24 orbitals, M=500 unless given); mixed: FP64 against FP32 / BF16 mixed-precision "
                         "Davidson solves from 5 seeded warm starts at the middle step")
    ap.add_argument("--partition", choices=["nc", "nc-cn"], default="nc",
                    help="NC MPO at every cut (default), or NC up to the middle cut and CN after it")
    ap.add_argument("--instances", type=int, default=16)
    ap.add_argument("--roots", type=int, default=1, help="apply workload: vectors per sigma-vector call")
    ap.add_argument("--kseg", type=int, default=0, help="split-K minimum segment (0 = default)")
    ap.add_argument("--no-t-merge", action="store_true",
                    help="keep one first-round intermediate per middle operator (no merged intermediates)")
    ap.add_argument("--bparts", type=int, default=1,
                    help="apply workload, FP64: also time the sigma-vector restricted to b = p (mod n) "
                         "for each of n middle-bond parts (one GPU's share of a sharded sigma)")
    ap.add_argument("--variant", type=int, default=None,
                    help="block-GEMM kernel variant (0 .. 6); default: chosen by the autotuner")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library defaults (or the given --variant/--kseg) instead of tuning")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sigma-vector would shard over the MPO middle-bond index, one all-reduce per call).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        if args.orbitals == 36 and args.bond_dim == 1000:
            args.orbitals, args.bond_dim = 16, 256
        bench_batch(args)
        return
    if args.workload == "sweep":
        if args.orbitals == 36 and args.bond_dim == 1000:
            args.orbitals, args.bond_dim = 24, 500
        if args.max_iter == 200:
            args.max_iter = 60
        bench_sweep(args)
        return

    import torch
    from paper_2310_03920_amd import _lib as X
    from paper_2310_03920_amd.dmrg import PRECISIONS, Davidson, split
    from paper_2310_03920_amd.engine import site_payload
    from paper_2310_03920_amd.mpo import build_mpo
    from synth import (bond_sector_tables, make_integrals, random_left_canonical_mps,
                       random_right_canonical_mps)
    from synth.blocks import random_psi

    X.lib()
    device = "cuda"
    K, N, M = args.orbitals, args.orbitals, args.bond_dim
    i = K // 2 - 1
    t0 = time.time()
    h, g = make_integrals(K, seed=0)
    mpo = build_mpo(h, g, switch=K // 2 if args.partition == "nc-cn" else None)
    bonds = bond_sector_tables(K, N, 0, M, model="gaussian", width=1.0)
    left = random_left_canonical_mps(bonds, 1)
    right = random_right_canonical_mps(bonds, 2)
    log(f"MPO + MPS set up in {time.time() - t0:.1f}s; D = {[len(mpo.cuts[k]) for k in (i, i + 1, i + 2)]}")
    Lenv, Renv = build_environments(X, mpo, bonds, left, right, i, device)

    tb = int(args.t_budget_gb * (1 << 30))
    opts, tune_s = plan_options(args, X, mpo, bonds, i, Lenv, Renv, tb, device)
    if args.workload == "apply":
        apply_only(args, X, mpo, bonds, i, Lenv, Renv, opts, tune_s, device)
        return
    if args.workload == "mixed":
        mixed_compare(args, X, mpo, bonds, i, Lenv, Renv, opts, tune_s, device)
        return
    t1 = time.time()
    plan = X.HeffPlan(bonds[i], bonds[i + 2], mpo.dq[i], mpo.dq[i + 1], mpo.dq[i + 2],
                      X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats),
                      X.MpoSite(mpo.sites[i + 1].rows, mpo.sites[i + 1].cols, mpo.sites[i + 1].mats), **opts)
    eplan = X.EnvPlan(0, bonds[i], bonds[i + 1], mpo.dq[i], mpo.dq[i + 1],
                      X.MpoSite(mpo.sites[i].rows, mpo.sites[i].cols, mpo.sites[i].mats), t_budget_bytes=tb,
                      kernel_variant=opts["kernel_variant"])
    plan_s = time.time() - t1
    plan.upload(device)
    eplan.upload(device)
    info, einfo = plan.info, eplan.info
    log(f"plans in {plan_s:.1f}s: psi {info.psi_nnz}, {info.flops_useful / 1e12:.3f} TFLOP/apply ({info.flops_apply / 1e12:.3f} executed), "
        f"tasks {info.n_tasks}, tiles {info.n_tiles}, chunks {info.n_chunks}, ws {info.ws_bytes / 1e9:.2f} GB")

    n = int(info.psi_nnz)
    rng = np.random.default_rng(3)
    lb, rb = X.Bond(bonds[i]), X.Bond(bonds[i + 2])
    psi0 = torch.from_numpy(X.pack_psi(lb, rb, random_psi(bonds[i], bonds[i + 2], rng))).to(device)
    diag = torch.empty(n, dtype=torch.float64, device=device)
    Lnew = torch.empty(int(einfo.out_nnz), dtype=torch.float64, device=device)
    dav = Davidson(n, args.kmax, device)
    fixed = dict(bonds[i + 1])
    ev = []

    ev32 = []
    v32 = torch.empty(n, dtype=torch.float32, device=device)
    s32 = torch.empty(n, dtype=torch.float32, device=device)

    def mv(v, out):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        plan.apply(Lenv, Renv, v, out)
        e.record()
        ev.append((s, e))

    low_apply = plan.apply_bf16 if args.mode == "bf16" else plan.apply_f32

    def mv32(v, out):
        X.convert_f64_f32(v, v32)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        low_apply(v32, s32)
        e.record()
        ev32.append((s, e))
        X.convert_f32_f64(s32, out)

    counts = {"f32": 0, "f64": 0}

    def site_step():
        plan.prepare(Lenv, Renv)
        plan.diag(Lenv, Renv, diag)
        if args.mode != "f64":
            plan.lower_f32(Lenv, Renv)
            theta, rnorm, n32, n64 = dav.solve_mixed(mv32, mv, psi0, diag, tol=args.tol, max_iter=args.max_iter,
                                                     **PRECISIONS[args.mode])
            counts["f32"] += n32
            counts["f64"] += n64
            nmv = n32 + n64
        else:
            theta, rnorm, nmv = dav.solve(mv, psi0, diag, tol=args.tol, max_iter=args.max_iter)
            counts["f64"] += nmv
        psi = X.unpack_psi(lb, rb, dav.x.cpu().numpy())
        nb, A, _, disc = split(psi, bonds[i], bonds[i + 2], M, 0, fixed=fixed)
        if nb != bonds[i + 1]:
            raise RuntimeError("truncation changed the bond table")
        eplan.update(Lenv, site_payload(bonds[i], bonds[i + 1], A, device), Lnew)
        return theta, rnorm, nmv, disc

    # warm start (untimed FP64 pre-solve) and the FP64 reference energy of this step
    plan.prepare(Lenv, Renv)
    plan.diag(Lenv, Renv, diag)
    t2 = time.time()
    _, r_pre, _ = dav.solve(mv, psi0, diag, tol=1e-12, max_iter=args.pre_iter)
    psi0 = dav.x.clone()
    e_ref, r_ref, n_ref = dav.solve(mv, psi0, diag, tol=1e-9, max_iter=600)
    ev.clear()
    log(f"warm start |r| = {r_pre:.2e}; reference E = {e_ref:.12f} (|r| {r_ref:.1e}, {n_ref} matvecs) "
        f"in {time.time() - t2:.1f}s")
    for _ in range(args.warmup):
        site_step()
    torch.cuda.synchronize()
    ev.clear()
    ev32.clear()
    counts["f32"] = counts["f64"] = 0
    times, res = [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res.append(site_step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    main_ev = ev32 if args.mode != "f64" else ev
    apply_ms = [s.elapsed_time(e) for s, e in main_ev]
    nmv = sum(r[2] for r in res)
    step_flops = [info.flops_prepare + r[2] * info.flops_useful + einfo.flops_apply for r in res]
    total_t = sum(times)
    value = sum(step_flops) / total_t / 1e9
    avg_apply = float(np.mean(apply_ms)) / 1e3
    achieved = info.flops_useful / avg_apply / 1e12
    peak = PEAKS[args.mode]
    theta, rnorm = res[-1][0], res[-1][1]
    # energy error of the mixed-precision step per block-product dtype (untimed, same warm
    # start and FP64 reference; in --mode f32 / bf16 the timed steps already are one)
    mixed = {}
    if args.mode == "f64":
        for md in ("f32", "bf16"):
            low = plan.apply_bf16 if md == "bf16" else plan.apply_f32

            def mv_low(v, out, low=low):
                X.convert_f64_f32(v, v32)
                low(v32, s32)
                X.convert_f32_f64(s32, out)

            try:
                plan.lower_f32(Lenv, Renv)
                t3 = time.perf_counter()
                th, rn, nl, nh = dav.solve_mixed(mv_low, mv, psi0, diag, tol=args.tol, max_iter=args.max_iter,
                                                 **PRECISIONS[md])
                torch.cuda.synchronize()
                mixed[md] = {"energy_err_vs_fp64": abs(th - e_ref), "rnorm": rn, "low_matvecs": nl,
                             "f64_matvecs": nh, "solve_s": time.perf_counter() - t3}
            except RuntimeError as exc:
                mixed[md] = {"error": str(exc)}
        plan.ws32 = plan.L32 = plan.R32 = None
        log(f"mixed-precision steps: {mixed}")
    traffic = (MEASURED_TRAFFIC.get((opts["kernel_variant"], opts["split_kseg_min"], opts["t_budget_bytes"],
                                     opts.get("t_merge_off", 0)))
               if (args.mode == "f64" and (K, M) == (36, 1000) and args.partition == "nc") else None)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total_t / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.mode,
        "data": "synthetic",
        "config": {
            "workload": f"two-site DMRG middle step (sites {i},{i + 1}) of a {K}-orbital ab initio chain, "
                        f"{N} electrons, 2Sz=0, M={M} (Gaussian sectors, width 1), integrals seed 0 "
                        f"(h ~ N(0,1)/sqrt(K), g = sum of 16 rank-1 terms of symmetric 0.1*N(0,1)), "
                        f"environments from a seeded random MPS, "
                        + ("NC-partition MPO" if args.partition == "nc" else f"NC-partition MPO up to cut {K // 2}, CN after"),
            "orbitals": K, "electrons": N, "bond_dim": M, "psi_nnz": n,
            "mpo_bond_dims": [len(mpo.cuts[k]) for k in (i, i + 1, i + 2)],
            "davidson": {"tol": args.tol, "max_iter": args.max_iter, "kmax": args.kmax, "matvecs_per_step": nmv / args.steps,
                         "warm_start_rnorm": r_pre, "reference_energy": e_ref, "reference_rnorm": r_ref,
                         "f32_matvecs_per_step": counts["f32"] / args.steps,
                         "f64_matvecs_per_step": counts["f64"] / args.steps, "precision": args.mode},
            "plan_build_s": plan_s, "chunks": int(info.n_chunks), "plan_opts": opts, "autotune_s": tune_s,
        },
        "heff_apply": {"ms": 1e3 * avg_apply, "tflop": info.flops_useful / 1e12,
                       "tflop_executed": info.flops_apply / 1e12, "bytes_algorithmic": info.bytes_apply,
                       "bytes_operands": 8.0 * (info.in_nnz + info.in2_nnz + 2 * info.psi_nnz),
                       "tflops": achieved, "launches": 2 * int(info.n_chunks)},
        "energy": theta,
        "rnorm": rnorm,
        "energy_err_vs_fp64": abs(theta - e_ref),
        "energy_err_vs_fp64_by_dtype": ({args.mode: abs(theta - e_ref)} if args.mode != "f64"
                                        else {"f64": abs(theta - e_ref),
                                              **{k: v.get("energy_err_vs_fp64") for k, v in mixed.items()}}),
        "mixed_precision_steps": mixed or None,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic[0] if traffic else None,
                     "traffic_source": traffic[1] if traffic else None,
                     "traffic_unit": "HBM bytes per sigma-vector (rocprofv3 FETCH_SIZE + WRITE_SIZE, stored)",
                     "kernel": ({"f32": "bsgemm<float> (all launches of one hx_heff_apply_f32)",
                                 "bf16": "bsgemm<float, BF16 products> (all launches of one hx_heff_apply_bf16)"
                                 }[args.mode] if args.mode != "f64"
                                else "bsgemm<double> (all launches of one hx_heff_apply)")},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mpo, bonds, i)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
