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


def test_ccd_leg(fake):
    tt, calls = fake
    wl = W.random_tensor((20, 15, 10), 300, 3)
    A0 = W.init_factors(wl.dims, 4, 1.0, 3)
    out = bench.compare_ccd(tt, None, A0, wl, 1e-5, "cpu")
    json.loads(json.dumps(out, allow_nan=False))
    assert set(out) == {"rmse_start", "als_ms", "als_rmse", "ccd_ms", "ccd_rmse"}
    assert calls.count("ccd_sweep") == 2 and calls.count("als_sweep") == 1
