#!/usr/bin/env python3
"""Benchmark of the completion hot path on one MI355X.

One step = one pass of the whole hot path over the resident tensor:
  * one ALS sweep: per mode MTTKRP of t (right-hand sides) and Solve Factor
    (Gram on matrix cores + FP64 Cholesky) -- Sections 2.2, 3.2, 3.4;
  * one preconditioned Gauss-Newton step with ``--cg`` CG iterations: the
    objective through the TTTP loss epilogue, the fused gradient adjoint,
    the block-diagonal preconditioner factorization, and per CG iteration one
    fused implicit GN matvec plus one preconditioner application -- Sections
    2.5 and 3.3.
The index (per-mode stable sort) is built once before timing and reported
separately.  ``value`` counts nonzero-rank products: m * R for every pass
over the nonzeros (TTTP, MTTKRP, gradient and GN-matvec passes, Gram passes)
divided by the step time.

Prints ONE JSON line.  Single GPU only.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MTTKRP+TTTP nnz·R/s, %HBM peak; ALS/GN sweep s, BF16 vs FP32 @ equal RMSE"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["ratings", "uniform"], default="ratings",
                   help="ratings: 100M-nonzero Zipf ratings tensor, ALS sweep + GN step; "
                        "uniform: 1.5B-nonzero 2^20-cubed tensor, TTTP + ALS sweep")
    p.add_argument("--R", type=int, default=None, help="rank (64 ratings, 32 uniform)")
    p.add_argument("--form", choices=["f32", "bf16"], default="f32")
    p.add_argument("--cg", type=int, default=2, help="CG iterations in the GN step")
    p.add_argument("--nnz", type=int, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 19)
    p.add_argument("--no-tune", dest="tune", action="store_false",
                   help="keep the default work partitions (no autotuner)")
    p.add_argument("--no-batching", dest="batching", action="store_false",
                   help="skip the graph-replay vs plain-launch comparison")
    p.add_argument("--form-sweeps", type=int, default=5,
                   help="ALS sweeps per storage form in the BF16-vs-FP32 comparison (0: skip)")
    p.add_argument("--no-ccd", dest="ccd", action="store_false",
                   help="ratings: skip the ALS-vs-CCD++ sweep comparison")
    p.add_argument("--poisson-iters", type=int, default=3,
                   help="ratings: GAM sweeps and GN steps of the Poisson log-link "
                        "comparison (0: skip)")
    p.add_argument("--gn-steps", type=int, default=3,
                   help="Gauss-Newton steps after the ALS sweeps of the forms comparison")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run a plain device copy of this size first (counter calibration)")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1910_02371_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload, src_hash):
    """HBM traffic per launch measured with rocprofv3 counters, if a committed
    summary for this kernel, workload and kernel source exists."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}|{workload}")
    except Exception:
        return None
    if not rec or rec.get("src_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single "
              "MI355X (multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1910_02371_amd import tt, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tt.lib()

    if args.calib_copy_mib:
        n = args.calib_copy_mib << 18
        xa = torch.ones(n, dtype=torch.float32, device=dev)
        xb = torch.empty_like(xa)
        torch.cuda.synchronize()
        xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb
    t0 = time.time()
    ratings = args.workload == "ratings"
    if ratings:
        wl = W.ratings(m=args.nnz or 100_000_000)
    else:
        wl = W.uniform(m=args.nnz or 1_500_000_000)
    gen_s = time.time() - t0
    log(f"generated {wl.name}: {wl.nnz} nnz in {gen_s:.1f}s")
    R = args.R or (64 if ratings else 32)
    lam = 1e-5      # least-squares ALS regularization (Section 5.6)
    lam_gn = 1e-3   # Gauss-Newton regularization of the paper's LS runs (Section 5.6)
    fdt_t = torch.float32 if args.form == "f32" else torch.bfloat16
    idx = [torch.as_tensor(i).to(dev) for i in wl.idx]
    t = torch.as_tensor(wl.t).to(dev)
    A0 = W.init_factors(wl.dims, R, float(np.mean(wl.t)), W.SEED_INIT + 2, dtype=np.float32)
    torch.cuda.synchronize()
    t0 = time.time()
    ix = tt.build_index(idx, wl.dims, t)
    torch.cuda.synchronize()
    index_s = time.time() - t0
    log(f"index built in {index_s:.2f}s")
    del idx, t  # the index holds its own sorted copies
    A = [torch.as_tensor(a).to(dev).to(fdt_t).contiguous() for a in A0]
    tuning = None
    if args.tune:
        # work-partition autotuner (cached per shape class; outside the timing)
        from paper_1910_02371_amd import autotune
        t0 = time.time()
        tuning = autotune.tune(tt, ix, A, R, lam, gn=ratings)
        tuning["seconds"] = time.time() - t0
        log(f"tuning {tuning['tuning']} ({'cached' if tuning['from_cache'] else 'measured'})")
    # the Gauss-Newton workspaces (and position map) only where the step has GN
    ix.reserve(R, tt.fdt_of([torch.empty(1, 1, dtype=fdt_t)]), gn="ls" if ratings else None)
    m = wl.nnz

    stream = torch.cuda.current_stream()
    names = []
    events = []

    def timed(name, fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        names.append(name)
        events.append((e0, e1))

    # per-mode right-hand sides and direction blocks for the separately timed
    # kernels of the step
    M = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in wl.dims]
    stats = torch.zeros(4, dtype=torch.float64, device=dev)

    out_m = None if ratings else torch.empty(m, dtype=torch.float32, device=dev)

    def step(record):
        run = timed if record else (lambda n, f: f())
        if not ratings:
            # model values for every nonzero, written in the index's mode-0
            # order (the library's sparse layout; the caller's COO order would
            # add a random scatter of m values)
            run("tttp", lambda: tt.tttp(ix, None, A, out=out_m, out_order=0))
        for n in range(3):
            # ALS update of mode n: Solve Factor with the MTTKRP(t) right-hand
            # side formed in the same pass over the nonzeros as the Gram
            run(f"als{n}", lambda n=n: tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, lam,
                                                       X=A[n]))
        if ratings:
            run("gn_step", lambda: tt.gn_step(ix, A, "ls", lam_gn, tol=5e-3, kmax=args.cg,
                                              stats=stats))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    tt.profile_enable(True)
    t0 = time.time()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.time() - t0
    tt.profile_enable(False)
    prof = tt.profile_report()
    ms_per_step = 1000.0 * wall / args.steps

    per = {}
    for nme, (e0, e1) in zip(names, events):
        per.setdefault(nme, []).append(e0.elapsed_time(e1))
    avg = {k: float(np.mean(v)) for k, v in per.items()}

    # nonzero passes of one step: ALS 3 MTTKRP + 3 Gram; GN step 1 TTTP +
    # 3 gradient + 3 Gram (preconditioner) + 3 GN-matvec per CG iteration;
    # the uniform workload: 1 TTTP + ALS
    passes = (6 + 1 + 3 + 3 + 3 * args.cg) if ratings else 7
    value = m * R * passes / (ms_per_step / 1000.0)

    # C-ABI calls of the step (HIP events on the launch stream)
    calls = {k: {"ms": v} for k, v in avg.items()}

    # dominant kernel: the library kernel with the largest total time over the
    # timed steps (library profiler: HIP events on the launch stream around
    # every launch, tagged with algorithmic bytes / flops per launch)
    dom, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    n_l = rec["launches"]
    per_ms = rec["ms"] / n_l
    src_hash = kernel_source_hash()
    wname = (f"{'ratings' if ratings else 'uniform'}{wl.dims[0]}x{wl.dims[1]}x{wl.dims[2]}"
             f"_m{m}_R{R}_{args.form}")
    traffic = traffic_from_profile(dom, wname, src_hash)
    # the Gram is a contraction: reported against the FP32 matrix-core peak
    # when its algorithmic intensity (flops per algorithmic byte) is above the
    # ridge point of that peak and the HBM bandwidth, else against HBM
    intensity = rec["flops"] / max(rec["bytes"], 1.0)
    if dom.startswith("gram") and intensity >= FP32_MFMA_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        achieved = rec["flops"] / n_l / (per_ms / 1e3) / 1e12
        roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved,
                    "peak": FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_MFMA_TFLOPS, "traffic": traffic,
                    "alg_flops_per_launch": rec["flops"] / n_l,
                    "alg_bytes_per_launch": rec["bytes"] / n_l, "launch_ms": per_ms,
                    "launches": n_l}
    else:
        achieved = rec["bytes"] / n_l / (per_ms / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": traffic, "alg_bytes_per_launch": rec["bytes"] / n_l,
                    "launch_ms": per_ms, "launches": n_l}
        # algorithmic bytes count every factor-row gather; when most of them
        # are served by L2 / Infinity Cache (measured HBM traffic below half
        # the algorithmic bytes, or a rate above the HBM peak) the rate is an
        # effective one
        roofline["effective"] = achieved > HBM_PEAK_GBS or (
            traffic is not None and traffic < 0.5 * rec["bytes"] / n_l)
    if traffic is not None:
        roofline["hbm_frac_measured"] = traffic / (per_ms / 1e3) / 1e9 / HBM_PEAK_GBS
    step_prof = {k: {"ms_per_step": v["ms"] / args.steps, "launches_per_step":
                     v["launches"] / args.steps,
                     "GBps_alg": v["bytes"] / v["ms"] / 1e6 if v["ms"] else None,
                     "TFLOPs_alg": v["flops"] / v["ms"] / 1e9 if v["ms"] else None}
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}

    batching = None
    if args.batching and ratings:
        batching = compare_batching(tt, ix, A, M, R, lam, lam_gn, args.cg, stats, dev)

    forms = None
    if args.form_sweeps > 0:
        forms = compare_forms(tt, ix, A0, wl, R, lam, args.form_sweeps, dev,
                              gn_steps=args.gn_steps if ratings else 0, lam_gn=lam_gn)

    poisson = None
    if args.poisson_iters > 0 and ratings:
        poisson = compare_poisson(tt, ix, wl, dev, args.poisson_iters)

    ccd = None
    if args.ccd and ratings:
        ccd = compare_ccd(tt, ix, A0, wl, lam, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, A0, R, lam, lam_gn, args.cpu_sample, passes, gn=ratings)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz*R/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.form,
        "data": "synthetic",
        "config": {
            "workload": (f"ratings-shaped {wl.dims[0]}x{wl.dims[1]}x{wl.dims[2]}, "
                         f"{m} distinct nonzeros, Zipf(1.1) mode degrees, values 1..5"
                         if ratings else
                         f"uniform {wl.dims[0]}x{wl.dims[1]}x{wl.dims[2]}, {m} nonzeros, "
                         f"planted rank 10 + N(0, 0.01^2)"),
            "step": ("ALS sweep (3 x [MTTKRP + Solve Factor], the MTTKRP right-hand "
                     "side formed in the Gram pass) + Gauss-Newton step" if ratings else
                     "TTTP (model values in the index's mode-0 order) + ALS sweep "
                     "(3 x [MTTKRP + Solve Factor], the MTTKRP right-hand side formed in "
                     "the Gram pass)"),
            "R": R, "factor_storage": args.form, "lambda": lam,
            "lambda_gn": lam_gn if ratings else None, "loss": "least squares",
            "cg_iterations": args.cg if ratings else None, "nnz_passes_per_step": passes,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "batching": batching,
        "poisson": poisson,
        "ccd": ccd,
        "tuning": tuning,
        "calls": calls,
        "step_kernels": step_prof,
        "index_build_s": index_s,
        "generate_s": gen_s,
        "src_hash": src_hash,
        "workload_key": wname,
    }
    print(json.dumps(out), flush=True)


def compare_batching(tt, ix, A, M, R, lam, lam_gn, cg, stats, dev, reps=3):
    """The step recorded once as a graph (tt_graph_begin/end) and replayed,
    against the same calls launched one by one, each also with persistent
    solve kernels (tuning solve_wgs = 8); and the same comparison for
    one ALS sweep on the 200^3 cube (40,000 nonzeros, R = 10, FP64), where
    launch overheads dominate.  Milliseconds per step / sweep (HIP events)."""
    import numpy as np
    import torch
    from paper_1910_02371_amd import workloads as W

    def timed_ms(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    info = [torch.empty(d, dtype=torch.int32, device=dev) for d in ix.dims]

    def step():
        for n in range(3):
            tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, lam, X=A[n], info=info[n])
        tt.gn_step(ix, A, "ls", lam_gn, tol=5e-3, kmax=cg, stats=stats)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plain = timed_ms(step, reps)
        g = tt.capture(step)
        g.launch()
        graph = timed_ms(g.launch, reps)
    torch.cuda.current_stream().wait_stream(side)
    g.close()
    # persistent solve kernels (a grid of 8 workgroups per compute unit that
    # strides over a batch's rows), launched one by one and as a graph
    torch.cuda.synchronize()
    t0 = ix.tuning()
    ix.tune(solve_wgs=8)
    ix.reserve(R, tt.fdt_of(A), gn="ls")
    with torch.cuda.stream(side):
        step()
        pers = timed_ms(step, reps)
        gp = tt.capture(step)
        gp.launch()
        pers_graph = timed_ms(gp.launch, reps)
    torch.cuda.current_stream().wait_stream(side)
    gp.close()
    torch.cuda.synchronize()
    ix.tune(**t0)
    ix.reserve(R, tt.fdt_of(A), gn="ls")

    wl = W.cube()
    Rc = 10
    Ac = [torch.as_tensor(a).to(dev) for a in
          W.init_factors(wl.dims, Rc, float(np.mean(wl.t)), W.SEED_INIT + 1, dtype=np.float64)]
    ixc = tt.build_index([torch.as_tensor(i).to(dev) for i in wl.idx], wl.dims,
                         torch.as_tensor(wl.t).to(dev))
    ixc.reserve(Rc, tt.TT_F64)
    infoc = torch.empty(sum(wl.dims), dtype=torch.int32, device=dev)
    with torch.cuda.stream(side):
        sweep = lambda: tt.als_sweep(ixc, Ac, 1e-5, infoc)
        sweep()
        plain_c = timed_ms(sweep, 20)
        gc = tt.capture(sweep)
        gc.launch()
        graph_c = timed_ms(gc.launch, 20)
    torch.cuda.current_stream().wait_stream(side)
    gc.close()
    return {"ratings_step_ms": {"plain": plain, "graph": graph, "persistent": pers,
                                "persistent_graph": pers_graph},
            "cube_als_sweep_ms": {"plain": plain_c, "graph": graph_c,
                                  "workload": "200^3, 40,000 nonzeros, R = 10, FP64"}}


def compare_forms(tt, ix, A0, wl, R, lam, sweeps, dev, gn_steps=0, lam_gn=1e-3, kmax=30):
    """ALS from the same FP32 start with FP32 and with BF16 factor storage:
    per-sweep wall time (HIP events) and training RMSE (TTTP loss epilogue,
    lambda = 0); then, from each form's ALS result, `gn_steps` Gauss-Newton
    steps (least squares, PCG with at most `kmax` iterations), timed the same
    way.  Equal RMSE means |RMSE_bf16 / RMSE_f32 - 1| <= 1% after the same
    number of sweeps (steps)."""
    import torch
    out = {}

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1)

    def rmse(A):
        return (tt.objective(ix, A, "ls", 0.0).item() / wl.nnz) ** 0.5

    for form, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        A = [torch.as_tensor(a).to(dev).to(dt).contiguous() for a in A0]
        info = torch.empty(sum(wl.dims), dtype=torch.int32, device=dev)
        rec = {"sweep_ms": [], "rmse": []}
        for _ in range(sweeps):
            rec["sweep_ms"].append(timed(lambda: tt.als_sweep(ix, A, lam, info)))
            rec["rmse"].append(rmse(A))
        if gn_steps:
            stats = torch.zeros(4, dtype=torch.float64, device=dev)
            rec["gn_ms"], rec["gn_rmse"] = [], []
            for _ in range(gn_steps):
                rec["gn_ms"].append(timed(lambda: tt.gn_step(ix, A, "ls", lam_gn, tol=5e-3,
                                                             kmax=kmax, stats=stats)))
                rec["gn_rmse"].append(rmse(A))
        out[form] = rec
    r32, r16 = out["f32"]["rmse"][-1], out["bf16"]["rmse"][-1]
    out["rmse_ratio_bf16_over_f32"] = r16 / r32
    out["equal_rmse_within_1pct"] = abs(r16 / r32 - 1.0) <= 0.01
    out["sweep_speedup_bf16"] = (sum(out["f32"]["sweep_ms"][1:]) /
                                 max(1e-9, sum(out["bf16"]["sweep_ms"][1:])))
    if gn_steps:
        g32, g16 = out["f32"]["gn_rmse"][-1], out["bf16"]["gn_rmse"][-1]
        out["gn_rmse_ratio_bf16_over_f32"] = g16 / g32
        out["gn_equal_rmse_within_1pct"] = abs(g16 / g32 - 1.0) <= 0.01
        out["gn_speedup_bf16"] = sum(out["f32"]["gn_ms"]) / max(1e-9, sum(out["bf16"]["gn_ms"]))
        out["gn_kmax"] = kmax
    return out


def compare_poisson(tt, ix, wl, dev, iters, R=10, lam=0.1, tol=1e-3, max_inner=5):
    """Poisson log-link completion of the same tensor, its values 1..5 read as
    counts, with Section 5.7's settings (R = 10, lambda = 0.1; alternating
    minimization inner Newton iterations to a relative step of 1e-3 or at
    most 5; PCG to 5e-3 or at most R iterations): from one start, `iters`
    generalized alternating-minimization sweeps and, separately, `iters`
    Gauss-Newton steps, each timed with HIP events, with the normalized loss
    (1/m) sum phi after each.  A first untimed call of each method on a copy
    allocates its workspaces."""
    import numpy as np
    import torch
    from paper_1910_02371_amd import workloads as W
    A0 = W.init_factors(wl.dims, R, float(np.log(np.mean(wl.t))), W.SEED_INIT + 3,
                        dtype=np.float32)
    m = wl.nnz

    def loss(A):
        v = tt.objective(ix, A, "poisson", 0.0).item() / m
        return v if np.isfinite(v) else None  # a diverged run stays valid JSON

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1), r

    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    run = {
        "gam": lambda A: tt.gam_sweep(ix, A, "poisson", lam, tol=tol, max_inner=max_inner),
        "gn": lambda A: tt.gn_step(ix, A, "poisson", lam, tol=5e-3, kmax=R, stats=stats),
    }
    out = {"R": R, "lambda": lam, "inner_tol": tol, "max_inner": max_inner, "cg_tol": 5e-3,
           "cg_kmax": R}
    for meth, fn in run.items():
        fn([torch.as_tensor(a).to(dev).contiguous() for a in A0])
        A = [torch.as_tensor(a).to(dev).contiguous() for a in A0]
        rec = {"ms": [], "loss": [loss(A)], "iterations": []}
        for _ in range(iters):
            ms, it = timed(lambda: fn(A))
            rec["ms"].append(ms)
            # GAM: Newton iterations per mode; GN: PCG iterations
            rec["iterations"].append(it if meth == "gam" else int(it[0].item()))
            rec["loss"].append(loss(A))
        out[meth] = rec
    # one Gauss-Newton product and one full Hessian product (the GN product
    # plus the phi' terms of the off-diagonal blocks, Section 2.5) at the
    # start point, with phi'' and phi' in each mode's order
    A = [torch.as_tensor(a).to(dev).contiguous() for a in A0]
    X = [torch.randn(d, R, device=dev) for d in wl.dims]
    w = [tt.tttp(ix, tt.INDEX_T, A, out_order=d, epi="d2phi", loss="poisson") for d in range(3)]
    g = [tt.tttp(ix, tt.INDEX_T, A, out_order=d, epi="dphi", loss="poisson") for d in range(3)]
    tt.newton_matvec(ix, w, g, A, X, 2 * lam)
    for name, fn in (("gn_matvec_ms", lambda: tt.gn_matvec(ix, w, A, X, 2 * lam)),
                     ("newton_matvec_ms", lambda: tt.newton_matvec(ix, w, g, A, X, 2 * lam))):
        out[name] = timed(fn)[0]
    return out


def compare_ccd(tt, ix, A0, wl, lam, dev):
    """One ALS sweep and one CCD++ sweep (Section 2.3: column-wise exact
    coordinate minimization, rank-1 MTTKRP + Solve Factor per column and
    mode) from the same FP32 start: time (HIP events) and training RMSE
    after the sweep.  A first untimed CCD++ sweep on a copy allocates its
    workspaces."""
    import torch

    def fresh():
        return [torch.as_tensor(a).to(dev).contiguous() for a in A0]

    def rmse(A):
        return (tt.objective(ix, A, "ls", 0.0).item() / wl.nnz) ** 0.5

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1)

    tt.ccd_sweep(ix, fresh(), lam)
    out = {"rmse_start": rmse(fresh())}
    for name, fn in (("als", tt.als_sweep), ("ccd", tt.ccd_sweep)):
        A = fresh()
        out[f"{name}_ms"] = timed(lambda: fn(ix, A, lam))
        out[f"{name}_rmse"] = rmse(A)
    return out


def cpu_baseline(wl, A0, R, lam, lam_gn, sample, passes, gn=True):
    """The FP64 oracle, as it stands, on a bounded sample: the first `sample`
    nonzeros (COO order is draw order, i.e. random) of the same tensor, full
    dimensions, same step composition (ALS sweep over the sampled rows, then
    objective, gradient, GN preconditioner Grams and CG matvecs)."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    import oracle as O

    idx = [i[:sample].astype(np.int64) for i in wl.idx]
    t = wl.t[:sample].astype(np.float64)
    A = [np.asarray(a, dtype=np.float64) for a in A0]
    ctx = threadpool_limits(1) if threadpool_limits else None
    t0 = time.time()
    try:
        ixs = O.build_index(idx, wl.dims)
        if not gn:
            O.tttp(idx, None, A)
        for n in range(3):
            Mn = O.mttkrp(idx, t, A, n, wl.dims[n])
            rows = ixs[n]["rows"]
            G = O.gram(idx, None, A, n, wl.dims[n], rows=rows)
            X, _ = O.solve_rows(G, Mn[rows], lam)
            A[n] = A[n].copy()
            A[n][rows] = X
        if gn:
            O.objective(idx, t, A, O.LOSS_LS, lam_gn)
            g = O.gradient(idx, t, A, O.LOSS_LS, lam_gn, wl.dims)
            for n in range(3):
                O.gram(idx, np.full(sample, 2.0), A, n, wl.dims[n], rows=ixs[n]["rows"])
            w = np.full(sample, 2.0)
            for _ in range((passes - 13) // 3):
                O.gn_matvec(idx, w, A, g, 2 * lam_gn, wl.dims)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    dt = time.time() - t0
    return {"value": sample * R * passes / dt, "unit": "nnz*R/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {sample} nonzeros (COO draw order) of the same tensor, full "
                      f"dimensions, one full step of the FP64 NumPy oracle; {dt:.1f}s"}


if __name__ == "__main__":
    main()
