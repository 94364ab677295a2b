"""Host logic of bench.py's comparison legs (CPU only): the Poisson GAM-vs-GN
leg and the ALS-vs-CCD++ leg run against a stand-in library object and
stand-in CUDA events, and their output is plain JSON (no GPU, no libtt)."""
import json
import os
import sys
import types

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1910_02371_amd import workloads as W  # noqa: E402


class _Event:
    def __init__(self, **kw):
        pass

    def record(self, *a):
        pass

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return 2.0


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(torch.cuda, "Event", _Event)
    calls = []

    def rec(name, ret):
        def f(*a, **k):
            calls.append(name)
            return ret(*a, **k)
        return f

    tt = types.SimpleNamespace(
        INDEX_T="t",
        objective=rec("objective", lambda ix, A, loss, lam: torch.tensor(0.5)),
        gam_sweep=rec("gam_sweep", lambda ix, A, loss, lam, tol, max_inner: [2, 1, 1]),
        gn_step=rec("gn_step", lambda ix, A, loss, lam, tol, kmax, stats: stats),
        tttp=rec("tttp", lambda ix, s, A, out_order, epi, loss: torch.zeros(3)),
        gn_matvec=rec("gn_matvec", lambda ix, w, A, X, lam2: X),
        newton_matvec=rec("newton_matvec", lambda ix, w, g, A, X, lam2: X),
        ccd_sweep=rec("ccd_sweep", lambda ix, A, lam: A),
        als_sweep=rec("als_sweep", lambda ix, A, lam: A))
    return tt, calls


def test_poisson_leg(fake):
    tt, calls = fake
    wl = W.random_tensor((20, 15, 10), 300, 3)
    wl.t[:] = np.round(np.abs(wl.t) * 4) + 1
    out = bench.compare_poisson(tt, None, wl, "cpu", 2)
    json.loads(json.dumps(out, allow_nan=False))
    assert out["R"] == 10 and out["lambda"] == 0.1 and out["cg_kmax"] == 10
    for meth in ("gam", "gn"):
        assert len(out[meth]["ms"]) == 2 and len(out[meth]["loss"]) == 3
    assert out["gam"]["iterations"] == [[2, 1, 1], [2, 1, 1]]
    assert out["gn"]["iterations"] == [0, 0]
    assert "newton_matvec_ms" in out and "gn_matvec_ms" in out
    # one untimed call per method, then the timed ones
    assert calls.count("gam_sweep") == 3 and calls.count("gn_step") == 3


def test_poisson_leg_reports_divergence_as_null(fake, monkeypatch):
    tt, _ = fake
    tt.objective = lambda ix, A, loss, lam: torch.tensor(float("inf"))
    wl = W.random_tensor((20, 15, 10), 300, 3)
    out = bench.compare_poisson(tt, None, wl, "cpu", 1)
    json.dumps(out, allow_nan=False)
    assert out["gn"]["loss"] == [None, None]


class _TunedIndex:
    """Stand-in for an index's tuning calls."""

    def __init__(self):
        self.cur = {"ccd_lds": -1}
        self.log = []

    def tuning(self):
        return dict(self.cur)

    def tune(self, **kw):
        self.log.append(kw)
        self.cur.update(kw)


@pytest.mark.parametrize("lds", [-1, 0])
def test_ccd_leg(fake, lds):
    """The CCD++ leg: keys, call counts, and the ccd_lds setting applied for
    the leg only (restored afterwards; no retuning when it is the index's)."""
    tt, calls = fake
    wl = W.random_tensor((20, 15, 10), 300, 3)
    A0 = W.init_factors(wl.dims, 4, 1.0, 3)
    ix = _TunedIndex()
    out = bench.compare_ccd(tt, ix, A0, wl, 1e-5, "cpu", lds)
    json.loads(json.dumps(out, allow_nan=False))
    assert set(out) == {"rmse_start", "als_ms", "als_rmse", "ccd_ms", "ccd_rmse", "ccd_lds"}
    assert out["ccd_lds"] == lds
    assert calls.count("ccd_sweep") == 2 and calls.count("als_sweep") == 1
    assert ix.log == ([] if lds == -1 else [{"ccd_lds": 0}, {"ccd_lds": -1}])
    assert ix.cur["ccd_lds"] == -1


def _rec(ms, launches, nbytes, flops):
    return {"launches": launches, "ms": ms, "bytes": nbytes, "flops": flops}


def test_roofline_prices_cache_served_gram_on_matrix_cores(monkeypatch):
    """A Gram launch whose algorithmic byte rate exceeds the HBM peak is a
    contraction bound by the matrix cores: frac is its flop rate over the
    FP32 peak, never an HBM fraction above 1."""
    monkeypatch.setattr(bench, "traffic_from_profile", lambda k, w: None)
    # 6.66 GB and 5.3e10 flop per launch in 0.478 ms
    r = bench.price_roofline("gram_heavy", _rec(0.478 * 10, 10, 6.66e10, 5.3e11), "w")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - 5.3e10 / 0.478e-3 / 1e12) < 1e-6
    assert 0 < r["frac"] <= 1 and r["effective_GBps"] > 8000


def test_roofline_measured_traffic_decides_the_bound(monkeypatch):
    rec = _rec(4.4 * 39, 39, 39 * 3.117e10, 39 * 1.2e11)
    # traffic equal to the algorithmic bytes: HBM binds
    monkeypatch.setattr(bench, "traffic_from_profile", lambda k, w: 3.13e10)
    r = bench.price_roofline("gram_heavy", rec, "w")
    assert r["bound"] == "hbm" and 0.85 < r["frac"] < 0.9 and r["traffic"] == 3.13e10
    # a quarter of them reach HBM: the matrix cores bind
    monkeypatch.setattr(bench, "traffic_from_profile", lambda k, w: 0.25 * 3.117e10)
    r = bench.price_roofline("gram_heavy", rec, "w")
    assert r["bound"] == "mfma" and r["frac"] <= 1


def test_roofline_streaming_kernel_above_peak_uses_measured_traffic(monkeypatch):
    rec = _rec(2.76, 1, 7.86e10, 1e10)  # 28 TB/s algorithmic: cache-served gathers
    monkeypatch.setattr(bench, "traffic_from_profile", lambda k, w: 1.78e10)
    r = bench.price_roofline("tttp", rec, "w")
    assert r["bound"] == "hbm" and r["effective"] and r["frac"] <= 1
    assert abs(r["achieved"] - 1.78e10 / 2.76e-3 / 1e9) < 1e-6
    monkeypatch.setattr(bench, "traffic_from_profile", lambda k, w: None)
    r = bench.price_roofline("tttp", rec, "w")
    assert r["frac"] is None and r["effective_GBps"] > 8000


def test_step_stats_and_time_to_rmse():
    s = bench.step_stats([10.0, 12.0, 11.0, 13.0])
    assert s["median"] == 11.5 and s["mean"] == 11.5 and s["n"] == 4
    assert abs(s["ci2sigma"] - 2 * np.std([10, 12, 11, 13], ddof=1)) < 1e-12
    t = bench.time_to_rmse([5, 5, 5], [0.3, 0.2, 0.1], [4, 4, 4], [0.3, 0.2, 0.1009])
    assert abs(t["target_rmse"] - 0.101) < 1e-12
    assert t["f32_ms"] == 15 and t["bf16_ms"] == 12 and t["bf16_sweeps"] == 3
    assert t["speedup_bf16"] == 15 / 12
    t = bench.time_to_rmse([5, 5], [0.3, 0.1], [4, 4], [0.3, 0.2])
    assert t["bf16_ms"] is None and t["speedup_bf16"] is None


def test_cpu_baseline_reports_both_thread_settings(monkeypatch):
    wl = W.random_tensor((30, 20, 10), 400, 5)
    A0 = W.init_factors(wl.dims, 4, 1.0, 3)
    out = bench.cpu_baseline(wl, A0, 4, 1e-5, 1e-3, 200, 7, gn=False, reps=2)
    json.loads(json.dumps(out, allow_nan=False))
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["value"] > 0
    assert len(out["runs_s"]) == 2 and out["one_core"]["value"] > 0
    assert "mean" in out["sample"] and out["mean_s"] > 0


def test_bench_refuses_several_gpus():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
