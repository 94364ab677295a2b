"""Autotuner of the work-partition parameters of an index (tile selection).

The kernels' results do not depend on these parameters beyond floating-point
summation order; their speed does, through occupancy (LDS per streaming
chunk), load balance (Gram task size, light/heavy threshold) and the width
of the workgroups that take heavy Gram tasks.  The paper fixes the analogous
choices from a memory model (the replication factor of its MTTKRP and the
row batches of Solve Factor, Sections 3.2 and 3.4); here they are measured.

Search: coordinate descent over KNOBS starting from the index's current
setting, one knob at a time in KNOBS order, keeping a candidate only if it
beats the best time so far by more than `min_gain`.  Each evaluation rebuilds
the index's partitions (tt_index_tune) and times `work`, a representative
call sequence (by default one ALS sweep's fused updates on every mode, plus
one Gauss-Newton matvec unless gn=False), with HIP events on the current
stream.

Results are cached in a JSON file keyed by factor dtype, rank and a shape
class of the tensor (log2 of the nonzero count and of the mean row degree of
every mode), so tensors of the same class reuse a setting without timing.
"""
import json
import math
import os

KNOBS = {
    "chunk": (512, 1024, 2048),
    "gram_piece": (2048, 4096, 8192),
    "gram_light": (256, 512, 1024),
    "gram_waves": (2, 4, 8),
    "solve_wgs": (0, 4, 8),
}

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1910_02371_amd",
                             "tuning.json")


def valid(t):
    return 0 <= t["gram_light"] <= t["gram_piece"]


def shape_key(dims, nnz, R, dtype_name):
    """Cache key: dtype, rank, round(log2 nnz), round(log2 mean degree) per mode."""
    lg = lambda x: int(round(math.log2(max(float(x), 1.0))))
    degs = "_".join(f"d{lg(nnz / max(int(d), 1))}" for d in dims)
    return f"{dtype_name}_R{R}_m{lg(nnz)}_{degs}"


def coordinate_descent(start, measure, knobs=KNOBS, min_gain=0.01):
    """Minimize measure(tuning) over knobs one at a time from `start`;
    returns (best tuning, best time, list of (tuning, time) evaluated)."""
    best = dict(start)
    best_t = measure(dict(best))
    trials = [(dict(best), best_t)]
    done = {tuple(sorted(best.items()))}
    for k, values in knobs.items():
        for v in values:
            cand = dict(best, **{k: v})
            key = tuple(sorted(cand.items()))
            if key in done or not valid(cand):
                continue
            done.add(key)
            t = measure(dict(cand))
            trials.append((dict(cand), t))
            if t < best_t * (1.0 - min_gain):
                best, best_t = cand, t
    return best, best_t, trials


def load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def default_work(tt, ix, A, R, lam, gn=True):
    """One ALS sweep's updates (Solve Factor with the MTTKRP right-hand side
    formed in the Gram pass) and (gn) one GN matvec, on scratch outputs (the
    factors are not changed)."""
    import torch
    dev = A[0].device
    dense = torch.float32 if A[0].dtype != torch.float64 else torch.float64
    X = [torch.empty_like(a) for a in A]
    info = [torch.empty(d, dtype=torch.int32, device=dev) for d in ix.dims]
    Y = [torch.empty((d, R), dtype=dense, device=dev) for d in ix.dims]
    Xd = [torch.rand((d, R), dtype=dense, device=dev) for d in ix.dims]

    def work():
        for n in range(len(A)):
            tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, lam, X=X[n], info=info[n])
        if gn:
            tt.gn_matvec(ix, None, A, Xd, 2 * lam, Y=Y)
    return work


def time_ms(work, reps):
    import torch
    work()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        work()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(tt, ix, A, R, lam=1e-5, work=None, reps=2, cache_path=DEFAULT_CACHE, retune=False,
         gn=True):
    """Pick the index's tuning (cached by shape class) and apply it; the
    default work includes a GN matvec when gn is set.
    Returns a report {"key", "tuning", "ms", "from_cache", "trials"}."""
    import torch
    dname = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[A[0].dtype]
    key = shape_key(ix.dims, ix.nnz, R, dname)
    cache = load_cache(cache_path) if cache_path else {}
    if not retune and key in cache:
        ix.tune(**cache[key]["tuning"])
        return {"key": key, "tuning": cache[key]["tuning"], "ms": cache[key]["ms"],
                "from_cache": True, "trials": []}
    work = work or default_work(tt, ix, A, R, lam, gn=gn)

    def measure(t):
        ix.tune(**t)
        return time_ms(work, reps)

    best, best_t, trials = coordinate_descent(ix.tuning(), measure)
    ix.tune(**best)
    if cache_path:
        cache[key] = {"tuning": best, "ms": best_t}
        save_cache(cache_path, cache)
    return {"key": key, "tuning": best, "ms": best_t, "from_cache": False,
            "trials": [{"tuning": t, "ms": ms} for t, ms in trials]}
