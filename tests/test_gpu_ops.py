"""GPU parity of the libtt primitives against the FP64 oracle, through the
C ABI (ctypes binding).  Small tensors spanning several work chunks, heavy
rows (> one chunk, > one Gram task), ragged ranks and every storage dtype."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1910_02371_amd import workloads as W
from gpu_helpers import (TAU, TAU_BF16_VS_F32, assert_close_abs, backward_error, dev_factor,
                         dev_idx, dev_vals, host, loss_abs, stored_factors, stored_values)

pytestmark = pytest.mark.gpu


def make_case(kind, seed=1):
    if kind == "uniform":
        wl = W.random_tensor((37, 41, 29), 3000, seed, rank=3)
    elif kind == "heavy":
        # mode-0 rows of ~5000 nonzeros: several streaming chunks and two
        # Gram tasks per row
        wl = W.random_tensor((3, 300, 200), 15000, seed, rank=2)
    elif kind == "zipf":
        rng = W.rng_for(seed)
        idx, _ = W.zipf_coords(rng, (3000, 400, 60), 60000, chunk=1 << 16)
        P = [rng.random((d, 4)) for d in (3000, 400, 60)]
        t = W._planted_values(idx, P)
        wl = W.Workload("zipf", (3000, 400, 60), idx, t, P)
    else:
        raise ValueError(kind)
    return wl


def factors(dims, R, seed, positive=False):
    rng = np.random.default_rng(seed)
    if positive:
        return [rng.random((d, R)) for d in dims]
    return [rng.standard_normal((d, R)) * 0.5 for d in dims]


_IX = {}


def get_index(tt, kind, form):
    key = (kind, form)
    if key not in _IX:
        wl = make_case(kind)
        ix = tt.build_index(dev_idx(wl.idx), wl.dims, dev_vals(wl.t, form))
        _IX[key] = (wl, ix)
    return _IX[key]


# ---------------------------------------------------------------- index ----
@pytest.mark.parametrize("case", ["uniform", "heavy", "zipf", "sorted", "reverse",
                                  "one_row", "empty_rows", "single"])
def test_index_bit_exact(gpu_lib, case):
    tt = gpu_lib
    rng = np.random.default_rng(5)
    if case in ("uniform", "heavy", "zipf"):
        wl = make_case(case)
        idx, dims = wl.idx, wl.dims
    else:
        dims = (50, 7, 300)
        m = 5000
        idx = [rng.integers(0, d, m) for d in dims]
        if case == "sorted":
            o = np.lexsort((idx[2], idx[1], idx[0]))
            idx = [a[o] for a in idx]
        elif case == "reverse":
            o = np.lexsort((idx[2], idx[1], idx[0]))[::-1]
            idx = [a[o] for a in idx]
        elif case == "one_row":
            idx[0][:] = 17
        elif case == "empty_rows":
            idx[2] = (idx[2] // 10) * 10
        elif case == "single":
            idx = [np.array([49]), np.array([0]), np.array([123])]
    ix = tt.build_index(dev_idx(idx), dims)
    ref = O.build_index(idx, dims)
    for n in range(3):
        ptr, perm, key, rows = ix.view(n)
        r = ref[n]
        assert np.array_equal(ptr.cpu().numpy(), r["ptr"]), f"ptr mode {n}"
        assert np.array_equal(perm.cpu().numpy(), r["perm"]), f"perm mode {n}"
        assert np.array_equal(key.cpu().numpy(), r["key"]), f"key mode {n}"
        assert np.array_equal(rows.cpu().numpy(), r["rows"]), f"rows mode {n}"
        for p in range(3):
            if p != n:
                assert np.array_equal(ix.other(n, p).cpu().numpy(), r["other"][p])


def test_index_range_error(gpu_lib):
    tt = gpu_lib
    idx = [np.array([0, 1, 2]), np.array([0, 5, 1]), np.array([0, 0, 0])]
    with pytest.raises(tt.TTError) as e:
        tt.build_index(dev_idx(idx), (3, 5, 1))
    assert e.value.status == -2


def test_index_empty(gpu_lib):
    tt = gpu_lib
    idx = [np.zeros(0, np.int32)] * 3
    ix = tt.build_index(dev_idx(idx), (4, 5, 6), dev_vals(np.zeros(0), "f32"))
    A = [dev_factor(np.ones((d, 4)), "f32") for d in (4, 5, 6)]
    Y = tt.mttkrp(ix, tt.INDEX_T, A, 1)
    assert torch.count_nonzero(Y).item() == 0
    _, s = tt.tttp(ix, tt.INDEX_T, A, out=False, epi="phi", want_sum=True)
    assert s.item() == 0.0
    # no nonzeros: the Gauss-Newton product is lambda2 * X
    X = [dev_factor(np.full((d, 4), 1.5), "f32") for d in (4, 5, 6)]
    Y = tt.gn_matvec(ix, None, A, X, 0.5, w_const=2.0)
    for y in Y:
        assert torch.all(y == 0.75).item()


# ----------------------------------------------------------------- TTTP ----
@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [1, 10, 13, 16, 32, 64])
@pytest.mark.parametrize("kind", ["uniform", "heavy"])
def test_tttp_parity(gpu_lib, form, R, kind):
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 100 + R)
    As = stored_factors(A64, form)
    s = stored_values(wl.t, form)
    A = [dev_factor(a, form) for a in A64]
    x = host(tt.tttp(ix, dev_vals(s, form), A))
    ref = O.tttp(wl.idx, s, As)
    ref_abs = O.tttp(wl.idx, np.abs(s), [np.abs(a) for a in As])
    assert_close_abs(x, ref, ref_abs, TAU[form], f"tttp {form} R={R}")
    if form == "bf16":
        ref32 = O.tttp(wl.idx, s, A64)
        abs32 = O.tttp(wl.idx, np.abs(s), [np.abs(a) for a in A64])
        assert_close_abs(x, ref32, abs32, TAU_BF16_VS_F32, "tttp bf16 vs unrounded")


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_tttp_orders_skips_and_sum(gpu_lib, form):
    tt = gpu_lib
    wl, ix = get_index(tt, "uniform", form)
    R = 8
    A64 = factors(wl.dims, R, 7)
    As = stored_factors(A64, form)
    s = stored_values(wl.t, form)
    A = [dev_factor(a, form) for a in A64]
    ref = O.tttp(wl.idx, s, As)
    ref_abs = O.tttp(wl.idx, np.abs(s), [np.abs(a) for a in As])
    for n in range(3):
        perm = O.build_index(wl.idx, wl.dims)[n]["perm"]
        # values in mode order, output in mode order
        xs = host(tt.tttp(ix, dev_vals(s[perm], form), A, s_order=n, out_order=n))
        assert_close_abs(xs, ref[perm], ref_abs[perm], TAU[form], f"tttp order {n}")
        # COO values, mode-order output
        xs = host(tt.tttp(ix, dev_vals(s, form), A, s_order=-1, out_order=n))
        assert_close_abs(xs, ref[perm], ref_abs[perm], TAU[form], f"tttp coo->{n}")
    # skipped mode (Section 3.3: the product runs over the provided modes)
    for skip in range(3):
        Ask = [None if n == skip else A[n] for n in range(3)]
        Aok = [None if n == skip else As[n] for n in range(3)]
        x = host(tt.tttp(ix, dev_vals(s, form), Ask))
        r = O.tttp(wl.idx, s, Aok)
        ra = O.tttp(wl.idx, np.abs(s), [None if a is None else np.abs(a) for a in Aok])
        assert_close_abs(x, r, ra, TAU[form], f"tttp skip {skip}")
    # Omega-hat and the FP64 sum
    x, tot = tt.tttp(ix, None, A, want_sum=True)
    r = O.tttp(wl.idx, None, As)
    ra = O.tttp(wl.idx, None, [np.abs(a) for a in As])
    assert_close_abs(host(x), r, ra, TAU[form], "tttp omega-hat")
    assert abs(tot.item() - r.sum()) <= TAU[form] * ra.sum()


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("loss", ["ls", "poisson"])
@pytest.mark.parametrize("epi", ["resid", "phi", "dphi", "d2phi"])
def test_tttp_epilogues(gpu_lib, form, loss, epi):
    tt = gpu_lib
    wl, ix = get_index(tt, "uniform", form)
    R = 16
    A64 = factors(wl.dims, R, 3, positive=True)
    A64 = [a * 0.4 for a in A64]
    As = stored_factors(A64, form)
    t = stored_values(np.abs(np.round(wl.t)), form) if loss == "poisson" else \
        stored_values(wl.t, form)
    tdev = dev_vals(t, form)
    ix2 = tt.build_index(dev_idx(wl.idx), wl.dims, tdev)
    A = [dev_factor(a, form) for a in A64]
    x, tot = tt.tttp(ix2, tt.INDEX_T, A, epi=epi, loss=loss, want_sum=True)
    m = O.tttp(wl.idx, None, As)
    m_abs = O.tttp(wl.idx, None, [np.abs(a) for a in As])
    L = O.LOSS_LS if loss == "ls" else O.LOSS_POISSON_LOG
    f = {"resid": lambda: t - m, "phi": lambda: O.phi(t, m, L),
         "dphi": lambda: O.dphi(t, m, L), "d2phi": lambda: O.d2phi(t, m, L)}[epi]()
    # the map on absolute values, the model value's error carried through
    # its slope (FP32 chain: model value <= 10 roundings, map <= 3)
    fabs = loss_abs(t, m, m_abs, L, epi)
    assert_close_abs(host(x), f, fabs, TAU[form], f"epi {epi}")
    assert abs(tot.item() - f.sum()) <= TAU[form] * fabs.sum()


# --------------------------------------------------------------- MTTKRP ----
@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [1, 10, 16, 32, 64])
@pytest.mark.parametrize("kind", ["uniform", "heavy", "zipf"])
def test_mttkrp_parity(gpu_lib, form, R, kind):
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 200 + R)
    As = stored_factors(A64, form)
    s = stored_values(wl.t, form)
    A = [dev_factor(a, form) for a in A64]
    for n in range(3):
        Y = host(tt.mttkrp(ix, tt.INDEX_T, A, n))
        ref = O.mttkrp(wl.idx, s, As, n, wl.dims[n])
        ref_abs = O.mttkrp(wl.idx, np.abs(s), [np.abs(a) for a in As], n, wl.dims[n])
        assert_close_abs(Y, ref, ref_abs, TAU[form], f"mttkrp {form} R={R} mode {n}")


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_mttkrp_weights_orders_accumulate(gpu_lib, form):
    tt = gpu_lib
    wl, ix = get_index(tt, "heavy", form)
    R = 12
    A64 = factors(wl.dims, R, 9)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(3)
    w = stored_values(rng.standard_normal(wl.nnz), form)
    for n in range(3):
        ref = O.mttkrp(wl.idx, w, As, n, wl.dims[n])
        ref_abs = O.mttkrp(wl.idx, np.abs(w), [np.abs(a) for a in As], n, wl.dims[n])
        Y = host(tt.mttkrp(ix, dev_vals(w, form), A, n, s_order=-1))
        assert_close_abs(Y, ref, ref_abs, TAU[form], f"coo weights mode {n}")
        perm = O.build_index(wl.idx, wl.dims)[n]["perm"]
        Y = host(tt.mttkrp(ix, dev_vals(w[perm], form), A, n, s_order=n))
        assert_close_abs(Y, ref, ref_abs, TAU[form], f"sorted weights mode {n}")
        # Omega-hat
        Y = host(tt.mttkrp(ix, None, A, n))
        r1 = O.mttkrp(wl.idx, None, As, n, wl.dims[n])
        ra = O.mttkrp(wl.idx, None, [np.abs(a) for a in As], n, wl.dims[n])
        assert_close_abs(Y, r1, ra, TAU[form], f"omega-hat mode {n}")
        # accumulate
        base = torch.full((wl.dims[n], R), 0.5, dtype=torch.float64 if form == "f64"
                          else torch.float32, device="cuda")
        Y = host(tt.mttkrp(ix, None, A, n, out=base, accumulate=True))
        assert_close_abs(Y, r1 + 0.5, ra + 0.5, TAU[form], f"accumulate mode {n}")


# ---------------------------------------------------------- solve factor ----
@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [1, 10, 16, 21, 32, 50, 64])
@pytest.mark.parametrize("kind", ["uniform", "heavy"])
def test_solve_factor_parity(gpu_lib, form, R, kind):
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 300 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    lam = 0.05
    rng = np.random.default_rng(R)
    for n in range(3):
        M = stored_values(rng.standard_normal((wl.dims[n], R)), form)
        Md = dev_vals(M, form)
        X, info = tt.solve_factor(ix, None, A, n, Md, lam)
        X = host(X)
        assert (info.cpu().numpy() == 0).all()
        G = O.gram(wl.idx, None, As, n, wl.dims[n])
        tau = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[form]
        be = backward_error(G, lam, X, M)
        assert be <= tau, f"backward error {be:.3e} (mode {n})"
        Xr, _ = O.solve_rows(G, M, lam)
        if form == "f64":
            np.testing.assert_allclose(X, Xr, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("form", ["f32", "bf16"])
@pytest.mark.parametrize("R", [21, 50, 64])
def test_solve_factor_weighted_lowp(gpu_lib, form, R):
    """Per-nonzero weights (the Gauss-Newton preconditioner's Gram) on rows
    with several Gram tasks, with and without vector factor loads."""
    tt = gpu_lib
    wl, ix = get_index(tt, "heavy", form)
    A64 = factors(wl.dims, R, 700 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(5 + R)
    w = stored_values(rng.random(wl.nnz) + 0.1, form)
    for n in range(3):
        M = stored_values(rng.standard_normal((wl.dims[n], R)), form)
        X, info = tt.solve_factor(ix, dev_vals(w, form), A, n, dev_vals(M, form), 0.05,
                                  w_order=-1)
        assert (info.cpu().numpy() == 0).all()
        G = O.gram(wl.idx, w, As, n, wl.dims[n])
        be = backward_error(G, 0.05, host(X), M)
        assert be <= {"f32": 1e-5, "bf16": 2e-2}[form], f"backward error {be:.3e} (mode {n})"


@pytest.mark.parametrize("form", ["f32", "bf16"])
@pytest.mark.parametrize("R", [16, 40, 64])
def test_solve_factor_not_spd_lowp(gpu_lib, form, R):
    """FP32/BF16 forms, whose one-task rows are factored in the solo-row
    kernels with L kept in the accumulator tiles: all-negative weights and
    lambda = 0 make every row's matrix negative semidefinite, so the first
    pivot fails: info equals the oracle's (LAPACK convention, 1 on every
    row), those rows of X are 0, and a synchronous call reports
    TT_ERR_NOT_SPD."""
    tt = gpu_lib
    wl, ix = get_index(tt, "uniform", form)
    A64 = factors(wl.dims, R, 900 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    wneg = -np.ones(wl.nnz)
    rng = np.random.default_rng(R)
    for n in range(3):
        M = stored_values(rng.standard_normal((wl.dims[n], R)), form)
        X, info = tt.solve_factor(ix, dev_vals(wneg, form), A, n, dev_vals(M, form), 0.0,
                                  w_order=-1)
        G = O.gram(wl.idx, wneg, As, n, wl.dims[n])
        _, ir = O.solve_rows(G, M, 0.0)
        assert (ir != 0).all()
        assert np.array_equal(info.cpu().numpy(), ir), f"mode {n}"
        assert (host(X) == 0).all(), f"mode {n}"
    M0 = stored_values(np.ones((wl.dims[0], R)), form)
    with pytest.raises(tt.TTError) as e:
        tt.solve_factor(ix, dev_vals(wneg, form), A, 0, dev_vals(M0, form), 0.0, w_order=-1,
                        sync=True)
    assert e.value.status == -5


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [10, 21, 64])
@pytest.mark.parametrize("kind", ["heavy", "zipf"])
def test_solve_factor_fused_rhs(gpu_lib, form, R, kind):
    """TT_RHS_MTTKRP: the ALS right-hand side MTTKRP(t) formed in the Gram
    pass (FP32/BF16; a separate MTTKRP for FP64) solves the oracle's normal
    equations (G + lambda I) x = MTTKRP(t)."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 800 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    s = stored_values(wl.t, form)
    lam = 0.05
    for n in range(3):
        X, info = tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, lam)
        assert (info.cpu().numpy() == 0).all()
        G = O.gram(wl.idx, None, As, n, wl.dims[n])
        M = O.mttkrp(wl.idx, s, As, n, wl.dims[n])
        tau = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[form]
        be = backward_error(G, lam, host(X), M)
        assert be <= tau, f"backward error {be:.3e} (mode {n})"
        if form == "f64":
            Xr, _ = O.solve_rows(G, M, lam)
            np.testing.assert_allclose(host(X), Xr, rtol=1e-8, atol=1e-10)


def _short_rows_tensor(R_counts, seed):
    """Mode-0 row i holds exactly R_counts[i] nonzeros (distinct coordinates
    in a 300 x 200 plane); every mode-0 row is one light Gram task."""
    rng = np.random.default_rng(seed)
    plane = 300 * 200
    keys = np.concatenate([i * plane + rng.choice(plane, size=k, replace=False)
                           for i, k in enumerate(R_counts)])
    idx = [a.astype(np.int32) for a in (keys // plane, (keys // 200) % 300, keys % 200)]
    return W.Workload("short_rows", (len(R_counts), 300, 200), idx,
                      rng.random(keys.size) * 4.0 + 1.0, None)


@pytest.mark.parametrize("form", ["f32", "bf16"])
@pytest.mark.parametrize("R,ld", [(64, 64), (40, 40), (50, 52)])
@pytest.mark.parametrize("lam", [0.05, 1e-5])
def test_solve_factor_short_rows(gpu_lib, form, R, ld, lam):
    """The fused least-squares update of rows with k <= 32 nonzeros at ranks
    above 32 solves the k x k system (c H H^T + lambda I) y = t and returns
    x = H^T y: every row count from 1 to 40 (both sides of 16 and 32),
    aligned, unaligned and padded factors; x meets the oracle's R x R
    normal equations (G + lambda I) x = MTTKRP(t) at the FP32 backward
    error, and (at lambda = 0.05) agrees with the oracle's solution."""
    tt = gpu_lib
    counts = list(range(1, 41)) * 2
    wl = _short_rows_tensor(counts, 71)
    ix = tt.build_index(dev_idx(wl.idx), wl.dims, dev_vals(wl.t, form))
    A64 = factors(wl.dims, R, 900 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    if ld != R:
        A = [_padded(a, ld) for a in A]
    s = stored_values(wl.t, form)
    X, info = tt.solve_factor(ix, None, A, 0, tt.RHS_MTTKRP, lam)
    assert (info.cpu().numpy() == 0).all()
    G = O.gram(wl.idx, None, As, 0, wl.dims[0])
    M = O.mttkrp(wl.idx, s, As, 0, wl.dims[0])
    tau = {"f32": 1e-5, "bf16": 2e-2}[form]
    be = backward_error(G, lam, host(X), M)
    assert be <= tau, f"backward error {be:.3e}"
    if lam > 1e-3:  # well conditioned: the solutions agree too
        Xr, _ = O.solve_rows(G, M, lam)
        err = np.linalg.norm(host(X) - Xr, axis=1) / np.maximum(np.linalg.norm(Xr, axis=1),
                                                                1e-30)
        bound = {"f32": 1e-3, "bf16": 5e-2}[form]
        assert err.max() <= bound, f"forward error {err.max():.3e} (row {err.argmax()})"


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [10, 32, 64])
@pytest.mark.parametrize("kind", ["heavy", "zipf"])
def test_solve_factor_model(gpu_lib, form, R, kind):
    """solve_factor_model: the ALS update equals solve_factor(RHS_MTTKRP) bit
    for bit (X and info, also in place), and the model values it returns
    (factors before the update, the mode's sorted order) equal the oracle's
    TTTP elementwise at tau (absolute form: the model on |A|)."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 700 + R)
    As = stored_factors(A64, form)
    ref = O.tttp(wl.idx, None, As)
    ref_abs = O.tttp(wl.idx, None, [np.abs(a) for a in As])
    lam = 0.05
    for n in range(3):
        A = [dev_factor(a, form) for a in A64]
        X0, info0 = tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, lam)
        X1, info1, model = tt.solve_factor_model(ix, A, n, lam)
        assert torch.equal(X0, X1) and torch.equal(info0, info1), f"mode {n}"
        perm = ix.view(n)[1].cpu().numpy()
        m_coo = np.empty(wl.nnz)
        m_coo[perm] = host(model)
        assert_close_abs(m_coo, ref, ref_abs, TAU[form], f"model values, mode {n}")
        # in place (X = A[n]): the same update and model values
        Xp, _, mp = tt.solve_factor_model(ix, A, n, lam, X=A[n])
        assert torch.equal(Xp, X1) and torch.equal(mp, model), f"in place, mode {n}"


def test_solve_factor_weights_and_info(gpu_lib):
    tt = gpu_lib
    form = "f64"
    wl, ix = get_index(tt, "uniform", form)
    R = 6
    A64 = factors(wl.dims, R, 11)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(2)
    w = rng.random(wl.nnz) + 0.2
    M = rng.standard_normal((wl.dims[1], R))
    X, info = tt.solve_factor(ix, dev_vals(w, form), A, 1, dev_vals(M, form), 0.3, w_order=-1)
    G = O.gram(wl.idx, w, A64, 1, wl.dims[1])
    Xr, _ = O.solve_rows(G, M, 0.3)
    np.testing.assert_allclose(host(X), Xr, rtol=1e-9, atol=1e-11)
    # negative weights making rows indefinite, lambda = 0: LAPACK info, x = 0
    wneg = -np.ones(wl.nnz)
    X, info = tt.solve_factor(ix, dev_vals(wneg, form), A, 1, dev_vals(M, form), 0.0,
                              w_order=-1)
    Gn = O.gram(wl.idx, wneg, A64, 1, wl.dims[1])
    _, ir = O.solve_rows(Gn, M, 0.0)
    assert np.array_equal(info.cpu().numpy(), ir)
    assert (host(X)[ir != 0] == 0).all()
    with pytest.raises(tt.TTError) as e:
        tt.solve_factor(ix, dev_vals(wneg, form), A, 1, dev_vals(M, form), 0.0, w_order=-1,
                        sync=True)
    assert e.value.status == -5


# ------------------------------------------------------ gradient / GN ----
@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("loss", ["ls", "poisson"])
@pytest.mark.parametrize("kind", ["uniform", "heavy"])
def test_gradient_and_objective(gpu_lib, form, loss, kind):
    tt = gpu_lib
    wl = make_case(kind)
    R = 16
    A64 = [0.5 * a for a in factors(wl.dims, R, 17, positive=True)]
    As = stored_factors(A64, form)
    L = O.LOSS_LS if loss == "ls" else O.LOSS_POISSON_LOG
    t = np.abs(np.round(wl.t)) if loss == "poisson" else wl.t
    t = stored_values(t, form)
    ix = tt.build_index(dev_idx(wl.idx), wl.dims, dev_vals(t, form))
    A = [dev_factor(a, form) for a in A64]
    lam = 0.1
    G = host(tt.gradient(ix, A, loss, lam))
    ref = O.gradient(wl.idx, t, As, L, lam, wl.dims)
    m = O.tttp(wl.idx, None, As)
    m_abs = O.tttp(wl.idx, None, [np.abs(a) for a in As])
    d1 = loss_abs(t, m, m_abs, L, "dphi")
    for d in range(3):
        ra = O.mttkrp(wl.idx, d1, [np.abs(a) for a in As], d, wl.dims[d]) + \
            2 * lam * np.abs(As[d])
        assert_close_abs(G[d], ref[d], ra, TAU[form], f"gradient mode {d}")
    f = tt.objective(ix, A, loss, lam).item()
    fr = O.objective(wl.idx, t, As, L, lam)
    fabs = np.sum(loss_abs(t, m, m_abs, L, "phi")) + lam * sum(np.sum(a * a) for a in As)
    assert abs(f - fr) <= TAU[form] * fabs


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("weights", ["const", "per_mode", "coo"])
@pytest.mark.parametrize("kind", ["uniform", "heavy", "zipf"])
def test_gn_matvec_parity(gpu_lib, form, weights, kind):
    """All three blocks of the product.  The scalar pass runs in the order of
    the mode with the most rows: mode 1 for the uniform and heavy cases,
    mode 0 for the Zipf case; the other blocks read its per-nonzero scalars
    through the index's position map."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    R = 16
    A64 = factors(wl.dims, R, 23)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(4)
    X64 = [stored_values(rng.standard_normal((d, R)), form) for d in wl.dims]
    Xd = [dev_vals(x, form) for x in X64]
    lam2 = 0.2
    if weights == "const":
        w = np.full(wl.nnz, 2.0)
        Y = tt.gn_matvec(ix, None, A, Xd, lam2, w_const=2.0)
    elif weights == "per_mode":
        w = stored_values(rng.random(wl.nnz) + 0.5, form)
        ixs = O.build_index(wl.idx, wl.dims)
        wd = [dev_vals(w[ixs[d]["perm"]], form) for d in range(3)]
        Y = tt.gn_matvec(ix, wd, A, Xd, lam2)
    else:
        w = stored_values(rng.random(wl.nnz) + 0.5, form)
        Y = tt.gn_matvec(ix, dev_vals(w, form), A, Xd, lam2, w_order=tt.ORDER_COO)
    Y = host(Y)
    ref = O.gn_matvec(wl.idx, w, As, X64, lam2, wl.dims)
    z_abs = O.jvp(wl.idx, [np.abs(a) for a in As], [np.abs(x) for x in X64])
    for d in range(3):
        ra = O.mttkrp(wl.idx, np.abs(w) * z_abs, [np.abs(a) for a in As], d, wl.dims[d]) + \
            lam2 * np.abs(X64[d])
        assert_close_abs(Y[d], ref[d], ra, TAU[form], f"gn mode {d}")


@pytest.mark.parametrize("form", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("R", [16, 21])
@pytest.mark.parametrize("kind", ["uniform", "heavy", "zipf"])
@pytest.mark.parametrize("g_order", ["per_mode", "coo"])
def test_newton_matvec_parity(gpu_lib, form, R, kind, g_order):
    """Full Hessian-vector product (GN product + phi' terms) for the Poisson
    log link at a random point: w = phi'' and g = phi' of the oracle's model
    values, stored at the value precision, against the oracle's product
    computed from t and the loss."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 41 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(6)
    X64 = [stored_values(rng.standard_normal((d, R)), form) for d in wl.dims]
    Xd = [dev_vals(x, form) for x in X64]
    L = O.LOSS_POISSON_LOG
    t = np.round(np.exp(np.abs(wl.t)))
    m = O.tttp(wl.idx, None, As)
    w = stored_values(O.d2phi(t, m, L), form)
    g = stored_values(O.dphi(t, m, L), form)
    ixs = O.build_index(wl.idx, wl.dims)
    wd = [dev_vals(w[ixs[d]["perm"]], form) for d in range(3)]
    if g_order == "per_mode":
        Y = tt.newton_matvec(ix, wd, [dev_vals(g[ixs[d]["perm"]], form) for d in range(3)],
                             A, Xd, 0.2)
    else:
        Y = tt.newton_matvec(ix, wd, dev_vals(g, form), A, Xd, 0.2, g_order=tt.ORDER_COO)
    Y = host(Y)
    # reference from the same stored w and g (t enters only through them)
    ref = O.gn_matvec(wl.idx, w, As, X64, 0.2, wl.dims)
    Aa, Xa = [np.abs(a) for a in As], [np.abs(x) for x in X64]
    z_abs = O.jvp(wl.idx, Aa, Xa)
    for d in range(3):
        ra = O.mttkrp(wl.idx, np.abs(w) * z_abs, Aa, d, wl.dims[d]) + 0.2 * Xa[d]
        for p in range(3):
            if p == d:
                continue
            Ap, Apa = list(As), list(Aa)
            Ap[p], Apa[p] = X64[p], Xa[p]
            ref[d] = ref[d] + O.mttkrp(wl.idx, g, Ap, d, wl.dims[d])
            ra = ra + O.mttkrp(wl.idx, np.abs(g), Apa, d, wl.dims[d])
        assert_close_abs(Y[d], ref[d], ra, TAU[form], f"newton mode {d}")
    if form == "f64" and R == 16 and g_order == "per_mode":
        # the same product from t and the loss, as the oracle defines it
        full = O.newton_matvec(wl.idx, t, As, X64, 0.2, wl.dims, L)
        for d in range(3):
            np.testing.assert_allclose(Y[d], full[d], rtol=1e-9, atol=1e-9 * np.abs(full[d]).max())


@pytest.mark.parametrize("form", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("R", [1, 13, 21, 64])
@pytest.mark.parametrize("kind", ["heavy", "zipf"])
def test_gn_matvec_ranks(gpu_lib, form, R, kind):
    """Ragged and full ranks (element and vector gather paths, one-lane
    rows) with per-mode weights; two calls in a row on the same index reuse
    its position map and scalar workspace."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    A64 = factors(wl.dims, R, 31 + R)
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    rng = np.random.default_rng(R)
    ixs = O.build_index(wl.idx, wl.dims)
    for call in range(2):
        X64 = [stored_values(rng.standard_normal((d, R)), form) for d in wl.dims]
        Xd = [dev_vals(x, form) for x in X64]
        w = stored_values(rng.random(wl.nnz) + 0.5, form)
        wd = [dev_vals(w[ixs[d]["perm"]], form) for d in range(3)]
        lam2 = 0.1 * (call + 1)
        Y = host(tt.gn_matvec(ix, wd, A, Xd, lam2))
        ref = O.gn_matvec(wl.idx, w, As, X64, lam2, wl.dims)
        z_abs = O.jvp(wl.idx, [np.abs(a) for a in As], [np.abs(x) for x in X64])
        for d in range(3):
            ra = O.mttkrp(wl.idx, np.abs(w) * z_abs, [np.abs(a) for a in As], d, wl.dims[d]) + \
                lam2 * np.abs(X64[d])
            assert_close_abs(Y[d], ref[d], ra, TAU[form], f"gn R={R} call {call} mode {d}")


# ------------------------------------------- padded leading dimension ----
def _padded(a, ld):
    """The factor `a` (device, I x R) stored in an I x ld buffer whose extra
    columns hold garbage (never read as part of the row)."""
    buf = torch.full((a.shape[0], ld), 3.0e4, dtype=a.dtype, device=a.device)
    buf[:, :a.shape[1]] = a
    return buf[:, :a.shape[1]]


@pytest.mark.parametrize("form", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("R", [10, 13, 21])
@pytest.mark.parametrize("kind", ["heavy", "zipf"])
def test_padded_ld_vector_path(gpu_lib, form, R, kind):
    """A rank that is not a multiple of the lane fragment (4 elements; 2 for
    FP64) with the factors' leading dimension padded to one: the streaming
    kernels read factor rows as whole fragments masked per column (the
    padding holds garbage), so TTTP, MTTKRP, the gradient, the GN product
    and the full Hessian product equal, bit for bit, the same calls on
    contiguous factors (element loads), and the oracle at tau."""
    tt = gpu_lib
    wl, ix = get_index(tt, kind, form)
    V = 2 if form == "f64" else 4
    ld = (R + V - 1) // V * V
    A64 = factors(wl.dims, R, 61 + R, positive=True)
    A64 = [0.6 * a for a in A64]
    As = stored_factors(A64, form)
    A = [dev_factor(a, form) for a in A64]
    Ap = [_padded(a, ld) for a in A]
    assert Ap[0].stride(0) == ld
    rng = np.random.default_rng(R)
    X64 = [stored_values(rng.standard_normal((d, R)), form) for d in wl.dims]
    Xd = [dev_vals(x, form) for x in X64]
    ixs = O.build_index(wl.idx, wl.dims)
    w = stored_values(rng.random(wl.nnz) + 0.5, form)
    wd = [dev_vals(w[ixs[d]["perm"]], form) for d in range(3)]
    g = stored_values(rng.standard_normal(wl.nnz), form)
    gd = [dev_vals(g[ixs[d]["perm"]], form) for d in range(3)]
    calls = {
        "tttp": lambda F: [tt.tttp(ix, tt.INDEX_T, F)],
        "mttkrp": lambda F: [tt.mttkrp(ix, tt.INDEX_T, F, n) for n in range(3)],
        "gradient": lambda F: tt.gradient(ix, F, "ls", 0.1),
        "gn": lambda F: tt.gn_matvec(ix, wd, F, Xd, 0.2),
        "newton": lambda F: tt.newton_matvec(ix, wd, gd, F, Xd, 0.2),
    }
    out = {}
    for name, fn in calls.items():
        a = [host(y) for y in fn(A)]
        b = [host(y) for y in fn(Ap)]
        for k, (ya, yb) in enumerate(zip(a, b)):
            assert np.array_equal(ya, yb), f"{name} block {k}: padded differs from contiguous"
        out[name] = b
    s = stored_values(wl.t, form)
    Aa = [np.abs(a) for a in As]
    m = O.tttp(wl.idx, None, As)
    m_abs = O.tttp(wl.idx, None, Aa)
    assert_close_abs(out["tttp"][0], s * m, np.abs(s) * m_abs, TAU[form], "padded tttp")
    for n in range(3):
        assert_close_abs(out["mttkrp"][n], O.mttkrp(wl.idx, s, As, n, wl.dims[n]),
                         O.mttkrp(wl.idx, np.abs(s), Aa, n, wl.dims[n]), TAU[form],
                         f"padded mttkrp mode {n}")
    ref = O.gn_matvec(wl.idx, w, As, X64, 0.2, wl.dims)
    z_abs = O.jvp(wl.idx, Aa, [np.abs(x) for x in X64])
    for d in range(3):
        ra = O.mttkrp(wl.idx, np.abs(w) * z_abs, Aa, d, wl.dims[d]) + 0.2 * np.abs(X64[d])
        assert_close_abs(out["gn"][d], ref[d], ra, TAU[form], f"padded gn mode {d}")
    ref = O.gradient(wl.idx, s, As, O.LOSS_LS, 0.1, wl.dims)
    d1 = loss_abs(s, m, m_abs, O.LOSS_LS, "dphi")
    for d in range(3):
        ra = O.mttkrp(wl.idx, d1, Aa, d, wl.dims[d]) + 0.2 * Aa[d]
        assert_close_abs(out["gradient"][d], ref[d], ra, TAU[form], f"padded gradient {d}")
    # the drivers on padded factors: one Gauss-Newton step and one
    # alternating-minimization sweep equal the contiguous runs bit for bit
    for drv in ("gn", "gam"):
        Ac = [a.clone() for a in A]
        Ad = [_padded(a, ld) for a in A]
        for F in (Ac, Ad):
            if drv == "gn":
                tt.gn_step(ix, F, "ls", 0.05, tol=1e-3, kmax=3)
            else:
                tt.gam_sweep(ix, F, "ls", 0.05, tol=0.0, max_inner=2)
        torch.cuda.synchronize()
        for d in range(3):
            assert torch.equal(Ac[d], Ad[d]), f"{drv} on padded factors, mode {d}"


# --------------------------------------------------------------- tuning ----
TUNINGS = [
    dict(chunk=512, gram_piece=2048, gram_light=256, gram_waves=2, solve_wgs=0, pcg_wgs=0,
         ccd_xcd=0, ccd_lds=0),
    dict(chunk=2048, gram_piece=8192, gram_light=1024, gram_waves=8, solve_wgs=1, pcg_wgs=2,
         ccd_xcd=1, ccd_lds=-1),
    dict(chunk=1024, gram_piece=1024, gram_light=0, gram_waves=4, solve_wgs=4, pcg_wgs=-1,
         ccd_xcd=-1, ccd_lds=-1),
]


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("kind", ["heavy", "zipf"])
def test_tuning_parity(gpu_lib, form, kind):
    """Every work-partition setting (chunk sizes, Gram task sizes, light and
    heavy thresholds, heavy workgroup widths, persistent solve grids) gives
    results within the same tolerances of the oracle: MTTKRP, TTTP sum, GN
    matvec and Solve Factor (given and fused right-hand sides), at aligned
    and unaligned ranks, in every storage form."""
    tt = gpu_lib
    wl = make_case(kind)
    ix = tt.build_index(dev_idx(wl.idx), wl.dims, dev_vals(wl.t, form))
    s = stored_values(wl.t, form)
    rng = np.random.default_rng(17)
    for tune in TUNINGS:
        ix.tune(**tune)
        assert ix.tuning() == tune
        for R in (64, 21):
            A64 = factors(wl.dims, R, 500 + R)
            As = stored_factors(A64, form)
            A = [dev_factor(a, form) for a in A64]
            for n in range(3):
                Y = host(tt.mttkrp(ix, tt.INDEX_T, A, n))
                ref = O.mttkrp(wl.idx, s, As, n, wl.dims[n])
                ref_abs = O.mttkrp(wl.idx, np.abs(s), [np.abs(a) for a in As], n, wl.dims[n])
                assert_close_abs(Y, ref, ref_abs, TAU[form], f"{tune} mttkrp R={R} mode {n}")
            _, tot = tt.tttp(ix, None, A, out=False, want_sum=True)
            m = O.tttp(wl.idx, None, As)
            m_abs = O.tttp(wl.idx, None, [np.abs(a) for a in As])
            assert abs(tot.item() - m.sum()) <= TAU[form] * m_abs.sum() + 1e-12
            X64 = [stored_values(rng.standard_normal((d, R)), form) for d in wl.dims]
            Yg = host(tt.gn_matvec(ix, None, A, [dev_vals(x, form) for x in X64], 0.1,
                                   w_const=2.0))
            refg = O.gn_matvec(wl.idx, np.full(wl.nnz, 2.0), As, X64, 0.1, wl.dims)
            z_abs = O.jvp(wl.idx, [np.abs(a) for a in As], [np.abs(x) for x in X64])
            for d in range(3):
                ra = O.mttkrp(wl.idx, 2.0 * z_abs, [np.abs(a) for a in As], d, wl.dims[d]) + \
                    0.1 * np.abs(X64[d])
                assert_close_abs(Yg[d], refg[d], ra, TAU[form], f"{tune} gn R={R} mode {d}")
            for n in range(3):
                M = stored_values(rng.standard_normal((wl.dims[n], R)), form)
                X, info = tt.solve_factor(ix, None, A, n, dev_vals(M, form), 0.05)
                assert (info.cpu().numpy() == 0).all()
                G = O.gram(wl.idx, None, As, n, wl.dims[n])
                be = backward_error(G, 0.05, host(X), M)
                assert be <= {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[form], \
                    f"{tune} solve R={R} mode {n}"
                X, info = tt.solve_factor(ix, None, A, n, tt.RHS_MTTKRP, 0.05)
                Mt = O.mttkrp(wl.idx, s, As, n, wl.dims[n])
                be = backward_error(G, 0.05, host(X), Mt)
                assert be <= {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[form], \
                    f"{tune} fused R={R} mode {n}"
