"""The C-ABI library loads and exports every entry point that include/tt.h
declares; host-side argument checks reject bad calls before touching the GPU
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tt.h")
LIB = os.path.join(ROOT, "paper_1910_02371_amd", "libtt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*"
                       r"([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_parses():
    names = declared_functions()
    for n in ["tt_build_index", "tt_index_destroy", "tt_index_view", "tttp", "mttkrp",
              "solve_factor", "gn_matvec", "tt_gradient", "tt_objective", "tt_als_sweep",
              "tt_gn_step", "tt_gam_sweep", "tt_ccd_sweep", "newton_matvec",
              "tt_last_error"]:
        assert n in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtt.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def test_binding_signatures_cover_header():
    from paper_1910_02371_amd import tt
    assert set(declared_functions()) == set(tt.SIGNATURES)


def test_host_argument_checks(lib):
    from paper_1910_02371_amd import tt
    L = tt.lib()
    # NULL index: rejected before any device work
    st = L.tttp(None, None, -1, None, 4, 4, 1, 0, 0, None, -1, None, None)
    assert st == -1
    assert b"index" in L.tt_last_error()
    st = L.mttkrp(None, None, -1, None, 4, 4, 1, 0, None, 0, None)
    assert st == -1
    st = L.solve_factor(None, None, -1, None, 4, 4, 1, 0, None, 0.0, None, None, 0, None)
    assert st == -1
    # bad order / dtype / nnz in tt_build_index
    dims = (ctypes.c_int64 * 5)(2, 2, 2, 2, 2)
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 5)()
    assert L.tt_build_index(5, dims, 0, arr, None, 1, 0, None, ctypes.byref(out)) == -1
    assert L.tt_build_index(3, dims, -1, arr, None, 1, 0, None, ctypes.byref(out)) == -1
    assert L.tt_build_index(3, dims, 0, arr, None, 7, 0, None, ctypes.byref(out)) == -1
    assert L.tt_index_destroy(None) == 0
    assert L.tt_version().startswith(b"libtt")
    # tuning and graph entry points validate on the host
    t = tt.Tuning(1024, 4096, 512, 4)
    assert L.tt_index_tune(None, ctypes.byref(t), None) == -1
    assert L.tt_index_get_tuning(None, ctypes.byref(t)) == -1
    assert L.tt_graph_begin(None) == -1
    assert b"stream" in L.tt_last_error()
    assert L.tt_graph_launch(None, None) == -1
    assert L.tt_graph_destroy(None) == 0
    assert L.tt_index_reserve(None, 8, 1, 0) == -1
    # the sweep drivers and the full Hessian product check their index first
    it = (ctypes.c_int32 * 3)()
    assert L.tt_gam_sweep(None, None, 4, 4, 1, 1, 0.1, 1e-3, 5, None, it, None) == -1
    assert b"index" in L.tt_last_error()
    assert L.tt_ccd_sweep(None, None, 4, 4, 1, 1e-5, None, None) == -1
    assert b"index" in L.tt_last_error()
    assert L.newton_matvec(None, None, -2, 2.0, None, -2, None, None, 4, 4, 1, 0.2,
                           None, None) == -1
    assert b"index" in L.tt_last_error()
