#!/usr/bin/env python3
"""Benchmark of the completion hot path on one MI355X.

Headline workload (``--workload uniform``, the default): the 2^20-cubed
tensor with 1.5 x 10^9 uniformly random nonzeros (one GPU's share of a
10^10-nonzero least-squares completion, Section 5.6), rank 32, FP32 factors.
One step = one TTTP over every nonzero (model values) + one ALS sweep, each
mode updated by Solve Factor with the MTTKRP(t) right-hand side formed in
the Gram pass (Sections 2.2, 3.2-3.4).  The BF16 factor-storage form is
compared with the FP32 form by ALS sweeps from the same start, at equal
training RMSE.

Secondary workload (``--secondary``, on by default; ``--workload ratings``
makes it the headline): the 10^8-nonzero Zipf ratings tensor at rank 64,
one step = one ALS sweep + one preconditioned Gauss-Newton step (Section
2.5), with the batching, BF16-form, Poisson (Section 5.7) and CCD++
(Section 2.3) comparison legs.

The index (per-mode stable sort) is built once before timing and reported
separately.  ``value`` counts nonzero-rank products: m * R for every pass
over the nonzeros the unfused method makes, divided by the step time.

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
# counters say the algorithmic bytes reach HBM when the measured traffic is at
# least this fraction of them
HBM_BINDS_FRAC = 0.8

# device code each profiled kernel is built from (the counters recorded in
# profiles/ are valid while these files are unchanged)
_SOLVE = ["solve_impl.h", "solve.hip", "solve_fused_f32.hip", "solve_fused_bf16.hip",
          "common.h"]
KERNEL_SOURCES = {
    "gram": _SOLVE,
    "cholesky": _SOLVE,
    "precond": _SOLVE,
    "stream": ["stream_impl.h", "stream_f32.hip", "stream_bf16.hip", "stream_f64.hip",
               "common.h"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["ratings", "uniform"], default="uniform",
                   help="uniform: 1.5B-nonzero 2^20-cubed tensor, TTTP + ALS sweep (headline); "
                        "ratings: 100M-nonzero Zipf ratings tensor, ALS sweep + GN step")
    p.add_argument("--R", type=int, default=None, help="rank (32 uniform, 64 ratings)")
    p.add_argument("--form", choices=["f32", "bf16"], default="f32")
    p.add_argument("--cg", type=int, default=2, help="CG iterations in the ratings GN step")
    p.add_argument("--nnz", type=int, default=None)
    p.add_argument("--no-secondary", dest="secondary", action="store_false",
                   help="uniform headline: skip the ratings-workload legs")
    p.add_argument("--secondary-steps", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=None,
                   help="nonzeros of the oracle's sample (default 2^16 uniform, 2^18 ratings)")
    p.add_argument("--cpu-reps", type=int, default=3,
                   help="timed oracle runs per thread setting (after one warm-up run)")
    p.add_argument("--no-tune", dest="tune", action="store_false",
                   help="keep the default work partitions (no autotuner)")
    p.add_argument("--no-batching", dest="batching", action="store_false",
                   help="skip the graph-replay vs plain-launch comparison")
    p.add_argument("--form-sweeps", type=int, default=5,
                   help="ALS sweeps per storage form in the BF16-vs-FP32 comparison (0: skip)")
    p.add_argument("--no-ccd", dest="ccd", action="store_false",
                   help="ratings: skip the ALS-vs-CCD++ sweep comparison")
    p.add_argument("--ccd-lds", type=int, choices=[-1, 0], default=-1,
                   help="ratings: the CCD++ sweep's ccd_lds tuning (LDS copies of small "
                        "record sets: -1 automatic, 0 off)")
    p.add_argument("--poisson-iters", type=int, default=3,
                   help="ratings: GAM sweeps and GN steps of the Poisson log-link "
                        "comparison (0: skip)")
    p.add_argument("--gn-steps", type=int, default=3,
                   help="Gauss-Newton steps after the ALS sweeps of the forms comparison")
    p.add_argument("--launch-bound", default=None, metavar="CASE:FORM",
                   help="only time the launch-bound GN step of CASE (small_gn or cube_gn) "
                        "in FORM (kernel_by_kernel, persistent_wgs1, persistent_wgs2, "
                        "automatic), launched one by one, and print its JSON (for a kernel "
                        "trace)")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run a plain device copy of this size first (counter calibration)")
    return p.parse_args(argv)


def kernel_family(kernel):
    if kernel.startswith("gram"):
        return "gram"
    if kernel.startswith("cholesky"):
        return "cholesky"
    if kernel == "precond_apply":
        return "precond"
    return "stream"


def kernel_source_hash(kernel=None):
    """Hash of the device sources of `kernel` (all of csrc/ when None)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1910_02371_amd", "csrc")
    files = sorted(os.listdir(d)) if kernel is None else KERNEL_SOURCES[kernel_family(kernel)]
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def profile_record(db_name, kernel, workload):
    """A committed counter record (profiles/<db_name>) for this kernel and
    workload, if it was measured on the current device sources."""
    path = os.path.join(ROOT, "profiles", db_name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}|{workload}")
    except Exception:
        return None
    if not rec or rec.get("src_hash") != kernel_source_hash(kernel):
        return None
    return rec


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, copy-kernel calibrated), or None."""
    rec = profile_record("traffic.json", kernel, workload)
    return rec.get("bytes_per_launch") if rec else None


def price_roofline(kernel, rec, workload, peak_gbs=HBM_PEAK_GBS, peak_tf=FP32_MFMA_TFLOPS):
    """Roofline entry of one kernel from the library profiler's record
    (launches, total ms, algorithmic bytes and flops over the timed steps).

    The bound is the one that binds: HBM when the kernel is a streaming
    (gather) kernel, or a Gram contraction whose measured HBM traffic is
    close to its algorithmic bytes; the FP32 matrix-core peak for a Gram
    whose gathers the caches serve (measured traffic well below the
    algorithmic bytes, or, unmeasured, an algorithmic byte rate above the
    HBM peak).  `frac` never exceeds what the bound allows: an algorithmic
    byte rate above the HBM peak is reported as `effective_GBps`, and the
    streaming kernels are then priced by their measured traffic."""
    n_l = rec["launches"]
    per_ms = rec["ms"] / n_l
    t = per_ms / 1e3
    alg_b = rec["bytes"] / n_l
    alg_f = rec["flops"] / n_l
    traffic = traffic_from_profile(kernel, workload)
    alg_rate = alg_b / t / 1e9
    out = {"kernel": kernel, "traffic": traffic, "alg_bytes_per_launch": alg_b,
           "alg_flops_per_launch": alg_f, "launch_ms": per_ms, "launches": n_l}
    if traffic is not None:
        out["hbm_frac_measured"] = traffic / t / 1e9 / peak_gbs
    contraction = kernel_family(kernel) == "gram"
    if traffic is not None:
        hbm_binds = traffic >= HBM_BINDS_FRAC * alg_b
    else:
        hbm_binds = alg_rate <= peak_gbs
    if contraction and not hbm_binds:
        ach = alg_f / t / 1e12
        out.update({"bound": "mfma", "achieved": ach, "peak": peak_tf, "unit": "TFLOP/s",
                    "frac": ach / peak_tf, "effective_GBps": alg_rate})
        cnt = profile_record("counters.json", kernel, workload)
        if cnt and "mfma_busy" in cnt:
            out["mfma_busy_measured"] = cnt["mfma_busy"]
        return out
    if alg_rate <= peak_gbs:
        out.update({"bound": "hbm", "achieved": alg_rate, "peak": peak_gbs, "unit": "GB/s",
                    "frac": alg_rate / peak_gbs, "effective": False})
        return out
    # algorithmic gathers beyond what HBM can deliver: most are cache hits
    meas = traffic / t / 1e9 if traffic is not None else None
    out.update({"bound": "hbm", "achieved": meas, "peak": peak_gbs, "unit": "GB/s",
                "frac": meas / peak_gbs if meas is not None else None, "effective": True,
                "effective_GBps": alg_rate})
    return out


def step_stats(ms):
    """Median, mean and the paper's 95% interval half-width (2 sigma) of
    per-step times (warm-up steps already dropped)."""
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    sd = float(a.std(ddof=1)) if len(a) > 1 else 0.0
    return {"median": float(np.median(a)), "mean": float(a.mean()), "ci2sigma": 2.0 * sd,
            "min": float(a.min()), "max": float(a.max()), "n": int(len(a))}


def time_steps(tt, step, steps, warmup):
    """`warmup` untimed steps, then exactly `steps` timed ones bracketed by
    device synchronizations (wall clock), with HIP events on the launch
    stream between consecutive steps and the library profiler on."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    tt.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.time()
    ev[0].record(stream)
    for k in range(steps):
        step(True)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    tt.profile_enable(False)
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return 1000.0 * wall / steps, per, tt.profile_report()


def kernel_table(prof, steps):
    return {k: {"ms_per_step": v["ms"] / steps, "launches_per_step": v["launches"] / steps,
                "GBps_alg": v["bytes"] / v["ms"] / 1e6 if v["ms"] else None,
                "TFLOPs_alg": v["flops"] / v["ms"] / 1e9 if v["ms"] else None}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}


class Leg:
    """One workload resident on the GPU: inputs, index (built once), tuned
    partitions and the step of the hot path timed on it."""

    def __init__(self, tt, W, workload, args, R=None, form="f32", tune=True, nnz=None):
        import numpy as np
        import torch
        self.tt, self.W, self.args = tt, W, args
        self.ratings = workload == "ratings"
        self.form = form
        dev = torch.device("cuda:0")
        self.dev = dev
        t0 = time.time()
        wl = W.ratings(m=nnz or 100_000_000) if self.ratings else \
            W.uniform(m=nnz or 1_500_000_000)
        self.gen_s = time.time() - t0
        log(f"generated {wl.name}: {wl.nnz} nnz in {self.gen_s:.1f}s")
        self.wl = wl
        self.R = R or (64 if self.ratings else 32)
        self.lam = 1e-5      # least-squares ALS regularization (Section 5.6)
        self.lam_gn = 1e-3   # Gauss-Newton regularization of the paper's LS runs (Section 5.6)
        self.fdt_t = torch.float32 if form == "f32" else torch.bfloat16
        idx = [torch.as_tensor(i).to(dev) for i in wl.idx]
        t = torch.as_tensor(wl.t).to(dev)
        self.A0 = W.init_factors(wl.dims, self.R, float(np.mean(wl.t)), W.SEED_INIT + 2,
                                 dtype=np.float32)
        torch.cuda.synchronize()
        t0 = time.time()
        self.ix = tt.build_index(idx, wl.dims, t)
        torch.cuda.synchronize()
        self.index_s = time.time() - t0
        log(f"index built in {self.index_s:.2f}s")
        del idx, t  # the index holds its own sorted copies
        self.A = [torch.as_tensor(a).to(dev).to(self.fdt_t).contiguous() for a in self.A0]
        self.tuning = None
        if tune:
            # work-partition autotuner (cached per shape class; outside the timing)
            from paper_1910_02371_amd import autotune
            t0 = time.time()
            self.tuning = autotune.tune(tt, self.ix, self.A, self.R, self.lam, gn=self.ratings)
            self.tuning["seconds"] = time.time() - t0
            log(f"tuning {self.tuning['tuning']} "
                f"({'cached' if self.tuning['from_cache'] else 'measured'})")
        # the Gauss-Newton workspaces (and position map) only where the step has GN
        self.ix.reserve(self.R, tt.fdt_of([torch.empty(1, 1, dtype=self.fdt_t)]),
                        gn="ls" if self.ratings else None)
        self.stats = torch.zeros(4, dtype=torch.float64, device=dev)
        self.out_m = None if self.ratings else torch.empty(wl.nnz, dtype=torch.float32,
                                                           device=dev)
        self.calls = {}
        # nonzero passes of one step: ALS 3 MTTKRP + 3 Gram; GN step 1 TTTP +
        # 3 gradient + 3 Gram (preconditioner) + 3 GN-matvec per CG iteration;
        # the uniform workload: 1 TTTP + ALS
        self.passes = (6 + 1 + 3 + 3 + 3 * args.cg) if self.ratings else 7
        self.wname = (f"{'ratings' if self.ratings else 'uniform'}"
                      f"{wl.dims[0]}x{wl.dims[1]}x{wl.dims[2]}_m{wl.nnz}_R{self.R}_{form}")

    def step(self, record):
        import torch
        tt, ix, A = self.tt, self.ix, self.A
        stream = torch.cuda.current_stream()

        def run(name, fn):
            if not record:
                fn()
                return
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            self.calls.setdefault(name, []).append((e0, e1))

        for n in range(3):
            # ALS update of mode n: Solve Factor with the MTTKRP(t) right-hand
            # side formed in the same pass over the nonzeros as the Gram
            if n == 0 and not self.ratings:
                # ... and, in mode 0's pass, the TTTP: the model value of every
                # nonzero for the factors at the start of the step, written in
                # the index's mode-0 order (the library's sparse layout; the
                # caller's COO order would add a random scatter of m values)
                run("tttp_als0", lambda: tt.solve_factor_model(ix, A, 0, self.lam, X=A[0],
                                                               model=self.out_m))
            else:
                run(f"als{n}", lambda n=n: tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP,
                                                           self.lam, X=A[n]))
        if self.ratings:
            run("gn_step", lambda: tt.gn_step(ix, A, "ls", self.lam_gn, tol=5e-3,
                                              kmax=self.args.cg, stats=self.stats))

    def measure(self, steps, warmup):
        import numpy as np
        self.calls = {}
        ms, per, prof = time_steps(self.tt, self.step, steps, warmup)
        m = self.wl.nnz
        value = m * self.R * self.passes / (ms / 1000.0)
        calls = {k: {"ms": float(np.mean([a.elapsed_time(b) for a, b in v]))}
                 for k, v in self.calls.items()}
        # dominant kernel: the library kernel with the largest total time over
        # the timed steps (library profiler: HIP events on the launch stream
        # around every launch, tagged with algorithmic bytes / flops)
        dom, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
        return {"ms_per_step": ms, "value": value, "step_ms": step_stats(per),
                "roofline": price_roofline(dom, rec, self.wname), "calls": calls,
                "step_kernels": kernel_table(prof, steps)}

    def close(self):
        import torch
        self.ix.close()
        self.A = None
        self.out_m = None
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single "
              "MI355X (multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

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

    if args.launch_bound:
        case, form = args.launch_bound.split(":")
        print(json.dumps(launch_bound_gn(tt, dev, reps=args.steps, cases=(case,),
                                         forms=(form,), graph=False)), flush=True)
        return

    leg = Leg(tt, W, args.workload, args, R=args.R, form=args.form, tune=args.tune,
              nnz=args.nnz)
    res = leg.measure(args.steps, args.warmup)
    log(f"{args.workload}: {res['ms_per_step']:.2f} ms per step "
        f"(median {res['step_ms']['median']:.2f})")
    wl, R = leg.wl, leg.R

    extra = {}
    if args.form_sweeps > 0:
        extra["forms"] = compare_forms(tt, leg.ix, leg.A0, wl, R, leg.lam, args.form_sweeps,
                                       dev, gn_steps=args.gn_steps if leg.ratings else 0,
                                       lam_gn=leg.lam_gn)
        log("forms leg done")
    if leg.ratings:
        extra.update(ratings_extras(tt, leg, args, dev))

    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample or (1 << 18 if leg.ratings else 1 << 16)
        cpu = cpu_baseline(wl, leg.A0, R, leg.lam, leg.lam_gn, sample, leg.passes,
                           gn=leg.ratings, reps=args.cpu_reps)
        log("cpu baseline done")

    secondary = None
    if args.secondary and not leg.ratings:
        head_meta = (leg.tuning, leg.index_s, leg.gen_s, leg.wname)
        leg.close()
        del leg
        sec = Leg(tt, W, "ratings", args, R=64, form="f32", tune=args.tune)
        r2 = sec.measure(args.secondary_steps, 2)
        log(f"ratings: {r2['ms_per_step']:.2f} ms per step")
        if args.form_sweeps > 0:
            r2["forms"] = compare_forms(tt, sec.ix, sec.A0, sec.wl, sec.R, sec.lam,
                                        args.form_sweeps, dev, gn_steps=args.gn_steps,
                                        lam_gn=sec.lam_gn)
        r2.update(ratings_extras(tt, sec, args, dev))
        r2.update({"workload": ratings_desc(sec), "step": step_desc(sec), "R": sec.R,
                   "nnz_passes_per_step": sec.passes, "steps": args.secondary_steps,
                   "warmup": 2, "tuning": sec.tuning, "index_build_s": sec.index_s,
                   "generate_s": sec.gen_s, "workload_key": sec.wname})
        secondary = {"ratings": r2}
        sec.close()
        tuning, index_s, gen_s, wname = head_meta
        cfg_leg = None
    else:
        tuning, index_s, gen_s, wname = leg.tuning, leg.index_s, leg.gen_s, leg.wname
        cfg_leg = leg

    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "nnz*R/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.form,
        "data": "synthetic",
        "config": {
            "workload": (ratings_desc(cfg_leg) if cfg_leg is not None and cfg_leg.ratings else
                         f"uniform {wl.dims[0]}x{wl.dims[1]}x{wl.dims[2]}, {wl.nnz} nonzeros, "
                         f"planted rank 10 + N(0, 0.01^2)"),
            "step": (step_desc(cfg_leg) if cfg_leg is not None else
                     "TTTP (model values in the index's mode-0 order) + ALS sweep "
                     "(3 x [MTTKRP + Solve Factor], the MTTKRP right-hand side formed in "
                     "the Gram pass; the TTTP formed in mode 0's pass from the same "
                     "gathered rows)"),
            "R": R, "factor_storage": args.form, "lambda": 1e-5,
            "lambda_gn": 1e-3 if args.workload == "ratings" else None,
            "loss": "least squares",
            "cg_iterations": args.cg if args.workload == "ratings" else None,
            "nnz_passes_per_step": 7 if args.workload == "uniform" else 6 + 1 + 9 + 3 * args.cg,
            "parallelism": "single GPU",
        },
        "step_ms": res["step_ms"],
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
        "tuning": tuning,
        "calls": res["calls"],
        "step_kernels": res["step_kernels"],
        "index_build_s": index_s,
        "generate_s": gen_s,
        "src_hash": kernel_source_hash(),
        "workload_key": wname,
    }
    out.update(extra)
    if secondary is not None:
        out["secondary"] = secondary
    print(json.dumps(out), flush=True)


def ratings_desc(leg):
    d = leg.wl.dims
    return (f"ratings-shaped {d[0]}x{d[1]}x{d[2]}, {leg.wl.nnz} distinct nonzeros, "
            f"Zipf(1.1) mode degrees, values 1..5")


def step_desc(leg):
    if leg.ratings:
        return ("ALS sweep (3 x [MTTKRP + Solve Factor], the MTTKRP right-hand side formed "
                f"in the Gram pass) + Gauss-Newton step ({leg.args.cg} CG iterations)")
    return ("TTTP (model values in the index's mode-0 order) + ALS sweep (3 x [MTTKRP + "
            "Solve Factor], the MTTKRP right-hand side formed in the Gram pass; the TTTP "
            "formed in mode 0's pass from the same gathered rows)")


def ratings_extras(tt, leg, args, dev):
    """Comparison legs run on the ratings tensor: launch batching, Poisson
    GAM vs GN, ALS vs CCD++."""
    out = {}
    if args.batching:
        out["batching"] = compare_batching(tt, leg.ix, leg.A, None, leg.R, leg.lam, leg.lam_gn,
                                           args.cg, leg.stats, dev)
        log("batching leg done")
    if args.poisson_iters > 0:
        out["poisson"] = compare_poisson(tt, leg.ix, leg.wl, dev, args.poisson_iters)
        log("poisson leg done")
    if args.ccd:
        out["ccd"] = compare_ccd(tt, leg.ix, leg.A0, leg.wl, leg.lam, dev, args.ccd_lds)
        log("ccd leg done")
    return out


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
                                  "workload": "200^3, 40,000 nonzeros, R = 10, FP64"},
            "gn_step_ms": launch_bound_gn(tt, dev)}


LB_FORMS = {"kernel_by_kernel": 0, "persistent_wgs1": 1, "persistent_wgs2": 2, "automatic": -1}


def launch_bound_gn(tt, dev, reps=10, kmax=30, cases=("small_gn", "cube_gn"),
                    forms=tuple(LB_FORMS), graph=True):
    """Launch-bound sizes: one Gauss-Newton step with kmax CG iterations
    (tolerance 0, so every step runs all of them) on (a) a 3 x 10^5-nonzero
    random tensor (1000^3, the size of Section 5.6's GN-vs-ALS comparison),
    R = 10, FP32, and (b) the 200^3 cube (40,000 nonzeros), R = 10, FP64;
    launched kernel by kernel, replayed as a graph, and with the CG
    iterations as one persistent kernel (pcg_wgs = 1 and 2 workgroups per
    compute unit, and the library's automatic choice; each launched and
    replayed as a graph); plus one ALS sweep of (a) launched and replayed.
    Milliseconds per call (HIP events)."""
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

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def plain_and_graph(fn):
        with torch.cuda.stream(side):
            fn()
            plain = timed_ms(fn, reps)
            if graph:
                g = tt.capture(fn)
                g.launch()
                replay = timed_ms(g.launch, reps)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        if not graph:
            return plain, None
        g.close()
        return plain, replay

    out = {}
    make = {"small_gn": lambda: ("1000^3, 300,000 uniform nonzeros, R = 10, FP32",
                                 W.random_tensor((1000, 1000, 1000), 300_000, W.SEED_DATA + 6,
                                                 rank=5, dtype=np.float32), np.float32,
                                 tt.TT_F32),
            "cube_gn": lambda: ("200^3 cube, 40,000 nonzeros, R = 10, FP64", W.cube(),
                                np.float64, tt.TT_F64)}
    for name in cases:
        desc, wl, npdt, fdt = make[name]()
        R = 10
        ix = tt.build_index([torch.as_tensor(i).to(dev) for i in wl.idx], wl.dims,
                            torch.as_tensor(wl.t).to(dev))
        A0 = W.init_factors(wl.dims, R, float(np.mean(wl.t)), W.SEED_INIT + 6, dtype=npdt)
        A = [torch.as_tensor(a).to(dev).contiguous() for a in A0]
        stats = torch.zeros(4, dtype=torch.float64, device=dev)
        res = {"workload": desc, "kmax": kmax, "tol": 0.0}
        step = lambda: tt.gn_step(ix, A, "ls", 1e-3, tol=0.0, kmax=kmax, stats=stats)
        for key in forms:
            ix.tune(pcg_wgs=LB_FORMS[key])
            ix.reserve(R, fdt, gn="ls")
            plain, replay = plain_and_graph(step)
            res[key] = {"plain": plain, "graph": replay}
        res["pcg_iterations"] = float(stats[0].item())
        ix.tune(pcg_wgs=0)
        if name == "small_gn" and graph:
            info = torch.empty(sum(wl.dims), dtype=torch.int32, device=dev)
            ix.reserve(R, fdt)
            plain, graph = plain_and_graph(lambda: tt.als_sweep(ix, A, 1e-5, info))
            res["als_sweep_ms"] = {"plain": plain, "graph": graph}
        ix.close()
        out[name] = res
    return out


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
    out["time_to_rmse"] = time_to_rmse(out["f32"]["sweep_ms"], out["f32"]["rmse"],
                                       out["bf16"]["sweep_ms"], out["bf16"]["rmse"])
    if gn_steps:
        g32, g16 = out["f32"]["gn_rmse"][-1], out["bf16"]["gn_rmse"][-1]
        out["gn_rmse_ratio_bf16_over_f32"] = g16 / g32
        out["gn_equal_rmse_within_1pct"] = abs(g16 / g32 - 1.0) <= 0.01
        out["gn_speedup_bf16"] = sum(out["f32"]["gn_ms"]) / max(1e-9, sum(out["bf16"]["gn_ms"]))
        out["gn_kmax"] = kmax
    return out


def time_to_rmse(ms32, rmse32, ms16, rmse16, slack=0.01):
    """Time each storage form takes to reach the FP32 form's final training
    RMSE within `slack` (equal RMSE): the summed sweep times up to the first
    sweep whose RMSE is at or below (1 + slack) * final FP32 RMSE; None if a
    form never reaches it."""
    target = (1.0 + slack) * rmse32[-1]

    def reach(ms, rm):
        acc = 0.0
        for k, (a, r) in enumerate(zip(ms, rm)):
            acc += a
            if r is not None and r <= target:
                return acc, k + 1
        return None, None

    t32, k32 = reach(ms32, rmse32)
    t16, k16 = reach(ms16, rmse16)
    return {"target_rmse": target, "f32_ms": t32, "f32_sweeps": k32, "bf16_ms": t16,
            "bf16_sweeps": k16,
            "speedup_bf16": (t32 / t16) if (t32 and t16) else None}


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
    # factors stored with their leading dimension padded to the 4-element
    # lane fragment (12 at R = 10), so the streaming kernels read whole
    # fragments
    ld = (R + 3) // 4 * 4

    def factors():
        out = []
        for a in A0:
            buf = torch.zeros((a.shape[0], ld), dtype=torch.float32, device=dev)
            buf[:, :R] = torch.as_tensor(a).to(dev)
            out.append(buf[:, :R])
        return out

    run = {
        "gam": lambda A: tt.gam_sweep(ix, A, "poisson", lam, tol=tol, max_inner=max_inner),
        "gn": lambda A: tt.gn_step(ix, A, "poisson", lam, tol=5e-3, kmax=R, stats=stats),
    }
    out = {"R": R, "ldA": ld, "lambda": lam, "inner_tol": tol, "max_inner": max_inner,
           "cg_tol": 5e-3, "cg_kmax": R}
    for meth, fn in run.items():
        fn(factors())
        A = factors()
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
    A = factors()
    X = [torch.randn(d, R, device=dev) for d in wl.dims]
    w = [tt.tttp(ix, tt.INDEX_T, A, out_order=d, epi="d2phi", loss="poisson") for d in range(3)]
    g = [tt.tttp(ix, tt.INDEX_T, A, out_order=d, epi="dphi", loss="poisson") for d in range(3)]
    tt.newton_matvec(ix, w, g, A, X, 2 * lam)
    for name, fn in (("gn_matvec_ms", lambda: tt.gn_matvec(ix, w, A, X, 2 * lam)),
                     ("newton_matvec_ms", lambda: tt.newton_matvec(ix, w, g, A, X, 2 * lam))):
        out[name] = timed(fn)[0]
    return out


def compare_ccd(tt, ix, A0, wl, lam, dev, ccd_lds=-1):
    """One ALS sweep and one CCD++ sweep (Section 2.3: column-wise exact
    coordinate minimization, rank-1 MTTKRP + Solve Factor per column and
    mode) from the same FP32 start: time (HIP events) and training RMSE
    after the sweep.  A first untimed CCD++ sweep on a copy allocates its
    workspaces.  ccd_lds: the index's tuning for the CCD++ sweeps (restored
    afterwards)."""
    import torch

    before = ix.tuning()["ccd_lds"]
    if ccd_lds != before:
        ix.tune(ccd_lds=ccd_lds)

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
    out = {"rmse_start": rmse(fresh()), "ccd_lds": ccd_lds}
    for name, fn in (("als", tt.als_sweep), ("ccd", tt.ccd_sweep)):
        A = fresh()
        out[f"{name}_ms"] = timed(lambda: fn(ix, A, lam))
        out[f"{name}_rmse"] = rmse(A)
    if ccd_lds != before:
        ix.tune(ccd_lds=before)
    return out


def cpu_info():
    """Host CPU model name and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    # the box grants this process a CPU share; OMP_NUM_THREADS states it
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return model, avail, (min(share, avail) if share > 0 else avail)


def cpu_baseline(wl, A0, R, lam, lam_gn, sample, passes, gn=True, reps=3):
    """The FP64 oracle, as it stands, on a bounded sample: the first `sample`
    nonzeros (COO order is draw order, i.e. random) of the same tensor, full
    dimensions, same step composition (uniform: TTTP + ALS sweep; ratings:
    ALS sweep, then objective, gradient, GN preconditioner Grams and CG
    matvecs).  One warm-up run, then `reps` timed runs (mean +- 2 sigma, the
    paper's convention), once with the BLAS/OpenMP pools on every CPU of the
    process's share and once on one thread."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    import oracle as O

    idx = [i[:sample].astype(np.int64) for i in wl.idx]
    t = wl.t[:sample].astype(np.float64)

    def one_step():
        A = [np.asarray(a, dtype=np.float64) for a in A0]
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

    def timed(threads):
        ctx = threadpool_limits(threads) if threadpool_limits else None
        ts = []
        try:
            for _ in range(reps + 1):
                t0 = time.time()
                one_step()
                ts.append(time.time() - t0)
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)
        ts = np.asarray(ts[1:])  # warm-up run dropped
        sd = float(ts.std(ddof=1)) if len(ts) > 1 else 0.0
        mean = float(ts.mean())
        return {"value": sample * R * passes / mean, "mean_s": mean, "ci2sigma_s": 2.0 * sd,
                "runs_s": [float(x) for x in ts]}

    model, avail, share = cpu_info()
    allc = timed(share)
    one = timed(1)
    return {"value": allc["value"], "unit": "nnz*R/s", "cores": share, "kind": "oracle",
            "sample": (f"first {sample} nonzeros (COO draw order) of the same tensor, full "
                       f"dimensions, one full step of the FP64 NumPy oracle; 1 warm-up + "
                       f"{reps} timed runs, mean {allc['mean_s']:.2f} s +- "
                       f"{allc['ci2sigma_s']:.2f} s (2 sigma) with the BLAS pool on {share} "
                       f"threads (its row loops are single-threaded NumPy)"),
            "mean_s": allc["mean_s"], "ci2sigma_s": allc["ci2sigma_s"], "runs_s": allc["runs_s"],
            "cpu_model": model, "cpus_visible": avail,
            "one_core": one}


if __name__ == "__main__":
    main()
