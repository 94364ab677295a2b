"""Thin ctypes binding of libtt (``include/tt.h``).

Argument marshalling only: every operation runs in the HIP kernels of
``libtt.so``.  Torch tensors provide device memory and the current HIP
stream.  Importing this module does not load the library; the first call
does, and raises ``RuntimeError`` if ``libtt.so`` has not been built.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtt.so")

TT_F64, TT_F32, TT_BF16 = 0, 1, 2
EPI = {"none": 0, "resid": 1, "phi": 2, "dphi": 3, "d2phi": 4}
LOSS = {"ls": 0, "poisson": 1, "poisson_log": 1}
ORDER_COO = -1
ORDER_PER_MODE = -2
INDEX_T = "t"          # selects the observed values held by the index
TT_SYNC = 1
RHS_MTTKRP = "mttkrp"  # solve_factor right-hand side = MTTKRP of the observed values
RESERVE_GN = 1
RESERVE_GN_POISSON = 2

STATUS = {0: "TT_OK", -1: "TT_ERR_INVALID_ARG", -2: "TT_ERR_INDEX_RANGE",
          -3: "TT_ERR_OOM", -4: "TT_ERR_HIP", -5: "TT_ERR_NOT_SPD",
          -6: "TT_ERR_UNSUPPORTED"}

# every entry point of include/tt.h with its ctypes signature
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_U32 = ctypes.c_uint32
_PP = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "tt_build_index": (_I, [_I, ctypes.POINTER(_I64), _I64, _PP, _P, _I, _U32, _P,
                            ctypes.POINTER(_P)]),
    "tt_index_destroy": (_I, [_P]),
    "tt_index_reserve": (_I, [_P, _I, _I, _U32]),
    "tt_index_tune": (_I, [_P, _P, _P]),
    "tt_index_get_tuning": (_I, [_P, _P]),
    "tt_index_view": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.POINTER(_P),
                           ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_I64)]),
    "tt_index_other": (_I, [_P, _I, _I, ctypes.POINTER(_P)]),
    "tttp": (_I, [_P, _P, _I, _PP, _I, _I64, _I, _I, _I, _P, _I, _P, _P]),
    "mttkrp": (_I, [_P, _P, _I, _PP, _I, _I64, _I, _I, _P, _I, _P]),
    "mttkrp_noalloc": (_I, [_P, _P, _I, _PP, _I, _I64, _I, _I, _P, _I, _P]),
    "solve_factor": (_I, [_P, _P, _I, _PP, _I, _I64, _I, _I, _P, _D, _P, _P, _U32, _P]),
    "solve_factor_model": (_I, [_P, _PP, _I, _I64, _I, _I, _D, _P, _P, _P, _P]),
    "gn_matvec": (_I, [_P, _P, _I, _D, _PP, _PP, _I, _I64, _I, _D, _PP, _P]),
    "newton_matvec": (_I, [_P, _P, _I, _D, _P, _I, _PP, _PP, _I, _I64, _I, _D, _PP, _P]),
    "tt_gradient": (_I, [_P, _PP, _I, _I64, _I, _I, _D, _PP, _P]),
    "tt_objective": (_I, [_P, _PP, _I, _I64, _I, _I, _D, _P, _P]),
    "tt_als_sweep": (_I, [_P, _PP, _I, _I64, _I, _D, _P, _P]),
    "tt_gn_step": (_I, [_P, _PP, _I, _I64, _I, _I, _D, _D, _I, _P, _P]),
    "tt_gam_sweep": (_I, [_P, _PP, _I, _I64, _I, _I, _D, _D, _I, _P, _P, _P]),
    "tt_ccd_sweep": (_I, [_P, _PP, _I, _I64, _I, _D, _P, _P]),
    "tt_graph_begin": (_I, [_P]),
    "tt_graph_end": (_I, [_P, ctypes.POINTER(_P)]),
    "tt_graph_launch": (_I, [_P, _P]),
    "tt_graph_destroy": (_I, [_P]),
    "tt_profile_enable": (_I, [_I]),
    "tt_profile_report": (_I, [ctypes.c_char_p, _I64, ctypes.POINTER(_I64)]),
    "tt_last_error": (ctypes.c_char_p, []),
    "tt_version": (ctypes.c_char_p, []),
}

_lib = None


class Tuning(ctypes.Structure):
    """tt_tuning: the work-partition parameters of an index."""
    _fields_ = [("chunk", ctypes.c_int32), ("gram_piece", ctypes.c_int32),
                ("gram_light", ctypes.c_int32), ("gram_waves", ctypes.c_int32),
                ("solve_wgs", ctypes.c_int32), ("pcg_wgs", ctypes.c_int32),
                ("ccd_xcd", ctypes.c_int32), ("ccd_lds", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class TTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libtt.so (once).  Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built: run `python -m paper_1910_02371_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise TTError(status, lib().tt_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def fdt_of(A):
    a = next(x for x in A if x is not None)
    return {torch.float64: TT_F64, torch.float32: TT_F32, torch.bfloat16: TT_BF16}[a.dtype]


def value_dtype(fdt):
    return torch.float64 if fdt == TT_F64 else torch.float32


def _rank_ld(A):
    a = next(x for x in A if x is not None)
    if a.dim() == 1:
        return 1, 1
    if a.stride(1) != 1:
        raise ValueError("factor rows must be contiguous")
    return a.shape[1], a.stride(0)


class Index:
    """Device index of a COO tensor (``tt_build_index``)."""

    def __init__(self, idx, dims, t=None, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.order = len(self.dims)
        self.nnz = int(idx[0].numel())
        self.has_t = t is not None
        self.vdt = TT_F64 if (t is not None and t.dtype == torch.float64) else TT_F32
        idx = [i.contiguous() for i in idx]
        for i in idx:
            if i.dtype != torch.int32 or not i.is_cuda:
                raise ValueError("indices must be int32 CUDA tensors")
        if t is not None:
            t = t.contiguous()
            if t.dtype not in (torch.float32, torch.float64):
                raise ValueError("values must be float32 or float64")
        dims_arr = (ctypes.c_int64 * self.order)(*self.dims)
        out = ctypes.c_void_p()
        self._h = None
        _check(lib().tt_build_index(self.order, dims_arr, self.nnz, _ptrs(idx), _ptr(t),
                                    self.vdt, 0, stream or _stream(), ctypes.byref(out)))
        self._h = out

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.tt_index_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self):
        t = Tuning()
        _check(lib().tt_index_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def tune(self, **kw):
        """Set work-partition parameters (chunk, gram_piece, gram_light,
        gram_waves, solve_wgs, pcg_wgs, ccd_xcd, ccd_lds; unspecified ones keep their value) and rebuild
        the partitions; reserve the workspace again afterwards."""
        cur = self.tuning()
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning parameters {sorted(unknown)}")
        cur.update(kw)
        t = Tuning(**cur)
        _check(lib().tt_index_tune(self._h, ctypes.byref(t), _stream()))

    def reserve(self, R, fdt, gn=None):
        """Size the workspace (needed before graph capture); gn = "ls" or
        "poisson" also sizes the Gauss-Newton step's workspace."""
        flags = {None: 0, "ls": RESERVE_GN, "poisson": RESERVE_GN | RESERVE_GN_POISSON}[gn]
        _check(lib().tt_index_reserve(self._h, R, fdt, flags))

    def view(self, mode):
        """(ptr int64[I+1], perm int32[m], key int32[m], rows int32[nrows]) as
        device tensors sharing the index's memory (read-only by contract)."""
        p, pe, k, r = (ctypes.c_void_p() for _ in range(4))
        nrows = ctypes.c_int64()
        _check(lib().tt_index_view(self._h, mode, ctypes.byref(p), ctypes.byref(pe),
                                   ctypes.byref(k), ctypes.byref(r), ctypes.byref(nrows)))
        I = self.dims[mode]
        return (_wrap(p.value, (I + 1,), torch.int64), _wrap(pe.value, (self.nnz,), torch.int32),
                _wrap(k.value, (self.nnz,), torch.int32),
                _wrap(r.value, (nrows.value,), torch.int32))

    def other(self, mode, other):
        p = ctypes.c_void_p()
        _check(lib().tt_index_other(self._h, mode, other, ctypes.byref(p)))
        return _wrap(p.value, (self.nnz,), torch.int32)


def _wrap(addr, shape, dtype):
    """Copy a device array owned by the library into a new torch tensor."""
    n = 1
    for s in shape:
        n *= s
    out = torch.empty(shape, dtype=dtype, device="cuda")
    if n:
        nbytes = n * out.element_size()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.restype = ctypes.c_int
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        torch.cuda.synchronize()
        rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(addr), nbytes, 3)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed: {rc}")
    return out


def build_index(idx, dims, t=None):
    return Index(idx, dims, t)


def _values(s):
    if s is None:
        return None
    if isinstance(s, str):
        if s != INDEX_T:
            raise ValueError(s)
        return ctypes.c_void_p(1)
    return _ptr(s)


def tttp(ix, s, A, out=None, s_order=ORDER_COO, out_order=ORDER_COO, epi="none",
         loss="ls", want_sum=False):
    """TTTP (Section 3.3) with an optional loss epilogue; returns ``out`` or
    ``(out, sum)``; ``out=False`` skips the per-nonzero output."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if out is None:
        out = torch.empty(ix.nnz, dtype=value_dtype(fdt), device="cuda")
    o = None if out is False else out
    ssum = torch.zeros((), dtype=torch.float64, device="cuda") if want_sum else None
    _check(lib().tttp(ix.handle, _values(s), s_order, _ptrs(A), R, ld, fdt, EPI[epi],
                      LOSS[loss], _ptr(o), out_order, _ptr(ssum), _stream()))
    return (o, ssum) if want_sum else o


def mttkrp(ix, s, A, mode, out=None, s_order=ORDER_COO, accumulate=False):
    """MTTKRP of mode ``mode`` (Section 3.2)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld([a for n, a in enumerate(A) if n != mode])
    if out is None:
        out = torch.empty((ix.dims[mode], R), dtype=value_dtype(fdt), device="cuda")
    _check(lib().mttkrp(ix.handle, _values(s), s_order, _ptrs(A), R, ld, fdt, mode, _ptr(out),
                        1 if accumulate else 0, _stream()))
    return out


def mttkrp_noalloc(ix, s, A, mode, out, s_order=ORDER_COO, accumulate=False):
    """MTTKRP of mode ``mode`` into the caller's ``out`` without any device
    allocation (carry scratch in the library's fixed per-device array);
    calls that overlap on one GPU race on that array."""
    fdt = fdt_of(A)
    R, ld = _rank_ld([a for n, a in enumerate(A) if n != mode])
    _check(lib().mttkrp_noalloc(ix.handle, _values(s), s_order, _ptrs(A), R, ld, fdt, mode,
                                _ptr(out), 1 if accumulate else 0, _stream()))
    return out


def solve_factor(ix, w, A, mode, rhs, lam, X=None, info=None, w_order=ORDER_COO,
                 sync=False):
    """Solve Factor (Section 3.4); returns (X, info).  ``rhs`` is an I x R
    array or RHS_MTTKRP (the ALS right-hand side MTTKRP(t), formed in the
    Gram pass)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld([a for n, a in enumerate(A) if n != mode])
    if X is None:
        # the library writes X with the factors' leading dimension
        dt = {TT_F64: torch.float64, TT_F32: torch.float32, TT_BF16: torch.bfloat16}[fdt]
        X = torch.empty((ix.dims[mode], ld), dtype=dt, device="cuda")[:, :R]
        ldx = ld
    else:
        ldx = X.stride(0)
        if ldx != ld:
            raise ValueError("X must share the factors' leading dimension")
    if info is None:
        info = torch.empty(ix.dims[mode], dtype=torch.int32, device="cuda")
    if isinstance(w, (list, tuple)):
        warr = _ptrs(w)
        wp = ctypes.cast(warr, ctypes.c_void_p)
        w_order = ORDER_PER_MODE
    else:
        warr = None
        wp = _values(w)
    rp = ctypes.c_void_p(2) if isinstance(rhs, str) and rhs == RHS_MTTKRP else _ptr(rhs)
    _check(lib().solve_factor(ix.handle, wp, w_order, _ptrs(A), R, ld, fdt, mode, rp,
                              float(lam), _ptr(X), _ptr(info), TT_SYNC if sync else 0,
                              _stream()))
    return X, info


def solve_factor_model(ix, A, mode, lam, X=None, info=None, model=None):
    """The ALS update of ``mode`` (solve_factor with RHS_MTTKRP) that also
    returns the model value of every nonzero for the factors before the
    update, in the index's mode-``mode`` sorted order; returns (X, info,
    model)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if X is None:
        dt = {TT_F64: torch.float64, TT_F32: torch.float32, TT_BF16: torch.bfloat16}[fdt]
        X = torch.empty((ix.dims[mode], ld), dtype=dt, device="cuda")[:, :R]
    elif X.stride(0) != ld:
        raise ValueError("X must share the factors' leading dimension")
    if info is None:
        info = torch.empty(ix.dims[mode], dtype=torch.int32, device="cuda")
    if model is None:
        model = torch.empty(ix.nnz, dtype=value_dtype(fdt), device="cuda")
    _check(lib().solve_factor_model(ix.handle, _ptrs(A), R, ld, fdt, mode, float(lam), _ptr(X),
                                    _ptr(info), _ptr(model), _stream()))
    return X, info, model


def gn_matvec(ix, w, A, X, lam2, Y=None, w_order=ORDER_PER_MODE, w_const=2.0):
    """Implicit Gauss-Newton matvec (Section 2.5); ``w`` is a list of per-mode
    weight arrays, a COO array, ``INDEX_T`` or None (constant ``w_const``)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if Y is None:
        Y = [torch.empty((d, R), dtype=value_dtype(fdt), device="cuda") for d in ix.dims]
    warr = None
    if isinstance(w, (list, tuple)):
        warr = _ptrs(w)
        wp = ctypes.cast(warr, ctypes.c_void_p)
        w_order = ORDER_PER_MODE
    else:
        wp = _values(w)
    _check(lib().gn_matvec(ix.handle, wp, w_order, float(w_const), _ptrs(A), _ptrs(X), R, ld,
                           fdt, float(lam2), _ptrs(Y), _stream()))
    return Y


def newton_matvec(ix, w, g, A, X, lam2, Y=None, w_order=ORDER_PER_MODE,
                  g_order=ORDER_PER_MODE, w_const=2.0):
    """Full Hessian-vector product (Section 2.5 with the phi' terms): the GN
    product with weights ``w`` (as in gn_matvec) plus the phi' terms with
    ``g`` = phi', a list of per-mode arrays or one COO array."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if Y is None:
        Y = [torch.empty((d, R), dtype=value_dtype(fdt), device="cuda") for d in ix.dims]
    keep = []

    def marshal(v, order):
        if isinstance(v, (list, tuple)):
            arr = _ptrs(v)
            keep.append(arr)
            return ctypes.cast(arr, ctypes.c_void_p), ORDER_PER_MODE
        return _values(v), order

    wp, w_order = marshal(w, w_order)
    gp, g_order = marshal(g, g_order)
    _check(lib().newton_matvec(ix.handle, wp, w_order, float(w_const), gp, g_order, _ptrs(A),
                               _ptrs(X), R, ld, fdt, float(lam2), _ptrs(Y), _stream()))
    return Y


def gradient(ix, A, loss, lam, G=None):
    """Gradient of the objective (Table 1 / Appendix A)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if G is None:
        G = [torch.empty((d, R), dtype=value_dtype(fdt), device="cuda") for d in ix.dims]
    _check(lib().tt_gradient(ix.handle, _ptrs(A), R, ld, fdt, LOSS[loss], float(lam),
                             _ptrs(G), _stream()))
    return G


def objective(ix, A, loss, lam, out=None):
    """f = sum phi + lam sum ||A_n||^2 as a float64 device scalar."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if out is None:
        out = torch.zeros((), dtype=torch.float64, device="cuda")
    _check(lib().tt_objective(ix.handle, _ptrs(A), R, ld, fdt, LOSS[loss], float(lam),
                              _ptr(out), _stream()))
    return out


def als_sweep(ix, A, lam, info=None):
    """One ALS sweep (Section 2.2), factors updated in place."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    _check(lib().tt_als_sweep(ix.handle, _ptrs(A), R, ld, fdt, float(lam), _ptr(info),
                              _stream()))
    return A


def gn_step(ix, A, loss, lam, tol=5e-3, kmax=30, stats=None):
    """One preconditioned Gauss-Newton step (Section 2.5), in place; returns
    the device stats [iterations, relative residual, initial residual,
    objective before the step]."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    if stats is None:
        stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    _check(lib().tt_gn_step(ix.handle, _ptrs(A), R, ld, fdt, LOSS[loss], float(lam),
                            float(tol), int(kmax), _ptr(stats), _stream()))
    return stats


def ccd_sweep(ix, A, lam, info=None):
    """One least-squares CCD++ sweep (Section 2.3), factors updated in place."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    _check(lib().tt_ccd_sweep(ix.handle, _ptrs(A), R, ld, fdt, float(lam), _ptr(info),
                              _stream()))
    return A


def gam_sweep(ix, A, loss, lam, tol=1e-3, max_inner=5, info=None, counts=True):
    """One generalized alternating-minimization sweep (Section 2.2, general
    loss; Section 5.7 inner stop rule), factors updated in place.  Returns
    the Newton iterations run per mode (host list), or None with
    counts=False (then the FP32 and BF16 forms never synchronize, and the
    call can be captured)."""
    fdt = fdt_of(A)
    R, ld = _rank_ld(A)
    iters = (ctypes.c_int32 * len(A))() if counts else None
    _check(lib().tt_gam_sweep(ix.handle, _ptrs(A), R, ld, fdt, LOSS[loss], float(lam),
                              float(tol), int(max_inner), _ptr(info), iters, _stream()))
    return list(iters) if counts else None


class Graph:
    """Library calls recorded once (tt_graph_begin/end) and replayed as one
    launch on the current stream."""

    def __init__(self, handle):
        self._h = handle

    def launch(self):
        _check(lib().tt_graph_launch(self._h, _stream()))

    def close(self):
        if self._h:
            lib().tt_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(fn):
    """Record the library calls that fn() makes on the current stream (not the
    null stream) into a Graph.  fn must allocate nothing: pass preallocated
    outputs and reserve the index workspace first."""
    s = _stream()
    _check(lib().tt_graph_begin(s))
    h = ctypes.c_void_p()
    try:
        fn()
    except BaseException:
        if lib().tt_graph_end(s, ctypes.byref(h)) == 0 and h.value:
            lib().tt_graph_destroy(h)
        raise
    _check(lib().tt_graph_end(s, ctypes.byref(h)))
    return Graph(h)


def profile_enable(on=True):
    """Start (clearing old records) or stop the library's kernel profiler."""
    _check(lib().tt_profile_enable(1 if on else 0))


def profile_report():
    """Per-kernel launches, total milliseconds, algorithmic bytes and flops."""
    import json
    need = ctypes.c_int64()
    _check(lib().tt_profile_report(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value + 16)
    _check(lib().tt_profile_report(buf, need.value + 16, ctypes.byref(need)))
    return json.loads(buf.value.decode())
