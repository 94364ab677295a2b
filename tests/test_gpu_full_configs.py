"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one by one (sampled
nonzeros for TTTP; sampled rows, with all their nonzeros, for MTTKRP,
Solve Factor, gradient and GN matvec) and through identities that hold at any
size.  Workloads: the 100M-nonzero ratings tensor (R = 64 and 16 FP32, R = 64
BF16), the 50M-nonzero Poisson counts tensor (R = 32) and the 1.5B-nonzero
uniform tensor (R = 32)."""
import gc
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_1910_02371_amd import workloads as W
from gpu_helpers import (TAU, TAU_BF16_VS_F32, assert_close_abs, host, loss_abs, rounded_abs,
                         stored_factors)

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


class Case:
    pass


def make_case(tt, wl, R, form, seed):
    c = Case()
    c.wl = wl
    c.R = R
    c.form = form
    vdt = torch.float64 if form == "f64" else torch.float32
    idx = [torch.as_tensor(i).cuda() for i in wl.idx]
    t = torch.as_tensor(wl.t).to(vdt).cuda()
    t0 = time.time()
    c.ix = tt.build_index(idx, wl.dims, t)
    torch.cuda.synchronize()
    say(f"index of {wl.name}: {time.time() - t0:.2f}s")
    del idx
    c.t_dev = t
    mean_model = float(np.mean(wl.t[:1 << 20]))
    if wl.meta.get("loss") == "poisson":
        mean_model = float(np.log(mean_model))
    A0 = W.init_factors(wl.dims, R, mean_model, seed, dtype=np.float32)
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[form]
    c.A = [torch.as_tensor(a).cuda().to(dt).contiguous() for a in A0]
    c.As = [a.to(torch.float64).cpu().numpy() if dt != torch.bfloat16 else
            a.float().to(torch.float64).cpu().numpy() for a in c.A]
    c.A0 = [a.astype(np.float64) for a in A0]
    c.t = wl.t.astype(np.float64) if form == "f64" else wl.t.astype(np.float32).astype(np.float64)
    return c


def sample_rows(idx_n, I_n, rng, max_nnz=400_000, k=4):
    cnt = np.bincount(idx_n, minlength=I_n)
    ok = np.flatnonzero((cnt > 0) & (cnt <= max_nnz))
    heavy = ok[np.argsort(cnt[ok])[-2:]]                 # heaviest rows under the cap
    light = ok[np.argsort(cnt[ok])[:1]]                  # a lightest row
    rand = rng.choice(ok, size=min(k, len(ok)), replace=False)
    return np.unique(np.concatenate([heavy, light, rand])), cnt


def subset(wl, n, rows):
    sel = np.flatnonzero(np.isin(wl.idx[n], rows))
    return [i[sel] for i in wl.idx], sel


# ----------------------------------------------------------- ratings ----
@pytest.fixture(scope="module")
def ratings_data():
    t0 = time.time()
    wl = W.ratings()
    say(f"ratings generated in {time.time() - t0:.1f}s")
    return wl


@pytest.fixture(scope="module")
def ratings64(gpu_lib, ratings_data):
    c = make_case(gpu_lib, ratings_data, 64, "f32", W.SEED_INIT + 2)
    yield c
    c.ix.close()
    del c
    gc.collect()
    torch.cuda.empty_cache()


def test_ratings_index_properties(gpu_lib, ratings64):
    """The stable sort at full size: keys non-decreasing, each permutation a
    bijection, ties in COO order, pointers equal to the key counts (these
    determine the stable argsort uniquely)."""
    c = ratings64
    for n in range(3):
        ptr, perm, key, rows = c.ix.view(n)
        perm = perm.cpu().numpy()
        key = key.cpu().numpy()
        ref_key = c.wl.idx[n][perm]
        assert np.array_equal(key, ref_key)
        assert np.all(np.diff(key) >= 0)
        assert np.array_equal(np.bincount(perm, minlength=c.wl.nnz), np.ones(c.wl.nnz))
        same = np.diff(key) == 0
        assert np.all(np.diff(perm)[same] > 0), "ties not in COO order"
        cnt = np.bincount(c.wl.idx[n], minlength=c.wl.dims[n])
        assert np.array_equal(np.diff(ptr.cpu().numpy()), cnt)
        del perm, key, ref_key


def test_ratings_tttp_and_identity(gpu_lib, ratings64):
    tt = gpu_lib
    c = ratings64
    rng = np.random.default_rng(1)
    x = tt.tttp(c.ix, c.t_dev, c.A)
    pos = rng.choice(c.wl.nnz, 20000, replace=False)
    sidx = [i[pos] for i in c.wl.idx]
    ref = O.tttp(sidx, c.t[pos], c.As)
    ra = O.tttp(sidx, np.abs(c.t[pos]), [np.abs(a) for a in c.As])
    assert_close_abs(host(x)[pos], ref, ra, TAU["f32"], "tttp sampled")
    # sum_e TTTP(t) = <A_n, MTTKRP_n(t)> for every mode (full size)
    _, tot = tt.tttp(c.ix, tt.INDEX_T, c.A, out=False, want_sum=True)
    _, tabs = tt.tttp(c.ix, tt.INDEX_T, [a.abs() for a in c.A], out=False, want_sum=True)
    for n in range(3):
        Y = tt.mttkrp(c.ix, tt.INDEX_T, c.A, n)
        ip = float((Y.double() * c.A[n].double()).sum().item())
        assert abs(ip - tot.item()) <= 1e-5 * tabs.item(), f"identity mode {n}"


def test_ratings_mttkrp_sampled_rows(gpu_lib, ratings64):
    tt = gpu_lib
    c = ratings64
    rng = np.random.default_rng(2)
    for n in range(3):
        Y = host(tt.mttkrp(c.ix, tt.INDEX_T, c.A, n))
        rows, cnt = sample_rows(c.wl.idx[n], c.wl.dims[n], rng)
        sidx, sel = subset(c.wl, n, rows)
        ref = O.mttkrp(sidx, c.t[sel], c.As, n, c.wl.dims[n])[rows]
        ra = O.mttkrp(sidx, np.abs(c.t[sel]), [np.abs(a) for a in c.As], n, c.wl.dims[n])[rows]
        assert_close_abs(Y[rows], ref, ra, TAU["f32"], f"mttkrp mode {n} rows {cnt[rows]}")


def test_ratings_solve_sampled_rows(gpu_lib, ratings64):
    """One ALS mode update at full size (Omega-hat Gram, M = MTTKRP(t),
    lambda = 1e-5): sampled rows have a small backward error against the
    oracle Gram and right-hand side."""
    tt = gpu_lib
    c = ratings64
    rng = np.random.default_rng(3)
    lam = 1e-5
    for n in range(3):
        M = tt.mttkrp(c.ix, tt.INDEX_T, c.A, n)
        X, info = tt.solve_factor(c.ix, None, c.A, n, M, lam)
        assert int((info != 0).sum().item()) == 0
        rows, cnt = sample_rows(c.wl.idx[n], c.wl.dims[n], rng, max_nnz=200_000)
        sidx, sel = subset(c.wl, n, rows)
        G = O.gram(sidx, None, c.As, n, c.wl.dims[n], rows=rows)
        Mr = O.mttkrp(sidx, c.t[sel], c.As, n, c.wl.dims[n])[rows]
        Xh = host(X)[rows]
        from gpu_helpers import backward_error
        be = backward_error(G, lam, Xh, Mr)
        assert be <= 1e-5, f"mode {n}: backward error {be:.2e} rows {cnt[rows]}"


def row_oracle(c, n, i, chunk=1 << 20):
    """The oracle's MTTKRP_n(t) row, its absolute form and the Gram of row i
    of mode n, summed over chunks of the row's nonzeros (each chunk is the
    sub-tensor of row i alone, its mode-n index mapped to 0)."""
    sel = np.flatnonzero(c.wl.idx[n] == i)
    R = c.R
    M, Ma, G = np.zeros(R), np.zeros(R), np.zeros((R, R))
    Aa = [np.abs(a) for a in c.As]
    for k in range(0, len(sel), chunk):
        part = sel[k:k + chunk]
        sub = [np.zeros(len(part), np.int64) if p == n else c.wl.idx[p][part]
               for p in range(3)]
        ts = c.t[part]
        M += O.mttkrp(sub, ts, c.As, n, 1)[0]
        Ma += O.mttkrp(sub, np.abs(ts), Aa, n, 1)[0]
        G += O.gram(sub, None, c.As, n, 1)[0]
    return M, Ma, G, len(sel)


def test_ratings_heaviest_rows(gpu_lib, ratings64):
    """Each mode's heaviest row (millions of nonzeros: hundreds of streaming
    pieces through the FP64 carries, thousands of Gram tasks through the
    FP64 task reductions): MTTKRP elementwise at tau, and Solve Factor with
    the given right-hand side and with the fused one (MTTKRP(t) formed in
    the Gram pass) by backward error against the oracle's Gram and
    MTTKRP."""
    from gpu_helpers import backward_error
    tt = gpu_lib
    c = ratings64
    lam = 1e-5
    for n in range(3):
        cnt = np.bincount(c.wl.idx[n], minlength=c.wl.dims[n])
        i = int(np.argmax(cnt))
        t0 = time.time()
        M, Ma, G, nz = row_oracle(c, n, i)
        say(f"mode {n} row {i}: {nz} nonzeros, oracle {time.time() - t0:.1f}s")
        Y = tt.mttkrp(c.ix, tt.INDEX_T, c.A, n)
        assert_close_abs(host(Y)[i], M, Ma, TAU["f32"], f"heaviest mttkrp mode {n} ({nz} nnz)")
        X, info = tt.solve_factor(c.ix, None, c.A, n, Y, lam)
        assert int(info[i].item()) == 0
        be = backward_error(G[None], lam, host(X)[i][None], host(Y)[i][None])
        assert be <= 1e-5, f"heaviest solve mode {n}: {be:.2e}"
        Xf, info = tt.solve_factor(c.ix, None, c.A, n, tt.RHS_MTTKRP, lam)
        assert int(info[i].item()) == 0
        be = backward_error(G[None], lam, host(Xf)[i][None], M[None])
        assert be <= 1e-5, f"heaviest fused solve mode {n}: {be:.2e}"
        del Y, X, Xf, info


def test_ratings_gradient_gn_sampled_rows(gpu_lib, ratings64):
    tt = gpu_lib
    c = ratings64
    rng = np.random.default_rng(4)
    lam = 1e-5
    G = host(tt.gradient(c.ix, c.A, "ls", lam))
    Xd = [torch.as_tensor(rng.standard_normal((d, c.R)).astype(np.float32)).cuda()
          for d in c.wl.dims]
    Xh = [x.double().cpu().numpy() for x in Xd]
    Y = host(tt.gn_matvec(c.ix, None, c.A, Xd, 2 * lam, w_const=2.0))
    for d in range(3):
        rows, cnt = sample_rows(c.wl.idx[d], c.wl.dims[d], rng, max_nnz=200_000, k=3)
        sidx, sel = subset(c.wl, d, rows)
        ts = c.t[sel]
        m = O.tttp(sidx, None, c.As)
        m_abs = O.tttp(sidx, None, [np.abs(a) for a in c.As])
        g = O.mttkrp(sidx, O.dphi(ts, m, O.LOSS_LS), c.As, d, c.wl.dims[d])[rows] + \
            2 * lam * c.As[d][rows]
        gabs = O.mttkrp(sidx, loss_abs(ts, m, m_abs, O.LOSS_LS, "dphi"),
                        [np.abs(a) for a in c.As], d, c.wl.dims[d])[rows] + \
            2 * lam * np.abs(c.As[d][rows])
        assert_close_abs(G[d][rows], g, gabs, TAU["f32"], f"gradient mode {d}")
        z = O.jvp(sidx, c.As, Xh)
        zabs = O.jvp(sidx, [np.abs(a) for a in c.As], [np.abs(x) for x in Xh])
        y = O.mttkrp(sidx, 2.0 * z, c.As, d, c.wl.dims[d])[rows] + 2 * lam * Xh[d][rows]
        yabs = O.mttkrp(sidx, 2.0 * zabs, [np.abs(a) for a in c.As], d, c.wl.dims[d])[rows] + \
            2 * lam * np.abs(Xh[d][rows])
        assert_close_abs(Y[d][rows], y, yabs, TAU["f32"], f"gn mode {d}")


def test_ratings_als_sweep_objective(gpu_lib, ratings64):
    tt = gpu_lib
    c = ratings64
    A = [a.clone() for a in c.A]
    f0 = tt.objective(c.ix, A, "ls", 1e-5).item()
    info = torch.empty(sum(c.wl.dims), dtype=torch.int32, device="cuda")
    tt.als_sweep(c.ix, A, 1e-5, info)
    f1 = tt.objective(c.ix, A, "ls", 1e-5).item()
    assert int((info != 0).sum().item()) == 0
    assert f1 < f0
    rmse = np.sqrt(tt.objective(c.ix, A, "ls", 0.0).item() / c.wl.nnz)
    say(f"ratings R=64 objective {f0:.4e} -> {f1:.4e}, RMSE {rmse:.4f}")


def test_ratings_r16(gpu_lib, ratings_data):
    tt = gpu_lib
    c = make_case(tt, ratings_data, 16, "f32", W.SEED_INIT + 3)
    try:
        rng = np.random.default_rng(5)
        x = host(tt.tttp(c.ix, c.t_dev, c.A))
        pos = rng.choice(c.wl.nnz, 20000, replace=False)
        sidx = [i[pos] for i in c.wl.idx]
        assert_close_abs(x[pos], O.tttp(sidx, c.t[pos], c.As),
                         O.tttp(sidx, np.abs(c.t[pos]), [np.abs(a) for a in c.As]),
                         TAU["f32"], "tttp R=16")
        for n in range(3):
            M = tt.mttkrp(c.ix, tt.INDEX_T, c.A, n)
            X, info = tt.solve_factor(c.ix, None, c.A, n, M, 1e-5)
            rows, cnt = sample_rows(c.wl.idx[n], c.wl.dims[n], rng, max_nnz=300_000)
            sidx, sel = subset(c.wl, n, rows)
            ref = O.mttkrp(sidx, c.t[sel], c.As, n, c.wl.dims[n])[rows]
            ra = O.mttkrp(sidx, np.abs(c.t[sel]), [np.abs(a) for a in c.As], n,
                          c.wl.dims[n])[rows]
            assert_close_abs(host(M)[rows], ref, ra, TAU["f32"], f"mttkrp R=16 mode {n}")
            G = O.gram(sidx, None, c.As, n, c.wl.dims[n], rows=rows)
            from gpu_helpers import backward_error
            assert backward_error(G, 1e-5, host(X)[rows], ref) <= 1e-5
    finally:
        c.ix.close()
        del c
        gc.collect()
        torch.cuda.empty_cache()


def test_ratings_bf16_r64_autograd_and_fd(gpu_lib, ratings_data):
    """BF16 factors, R = 64: the CPLoss adjoint at full size against the
    oracle gradient on sampled rows (same rounded factors: 1e-5 of the
    absolute expression; unrounded FP32 factors: 2e-2), and on a 1,000-nonzero
    subsample the FP64 form's gradient against central finite differences of
    its own objective."""
    from paper_1910_02371_amd.autograd import cp_loss
    tt = gpu_lib
    c = make_case(tt, ratings_data, 64, "bf16", W.SEED_INIT + 2)
    try:
        lam = 1e-5
        A = [a.clone().requires_grad_(True) for a in c.A]
        f = cp_loss(c.ix, A, "ls", lam)
        f.backward()
        rng = np.random.default_rng(6)
        for d in range(3):
            rows, cnt = sample_rows(c.wl.idx[d], c.wl.dims[d], rng, max_nnz=200_000, k=3)
            sidx, sel = subset(c.wl, d, rows)
            ts = c.t[sel]
            for As, tau in ((c.As, TAU["bf16"]), (c.A0, TAU_BF16_VS_F32)):
                m = O.tttp(sidx, None, As)
                m_abs = O.tttp(sidx, None, [np.abs(a) for a in As])
                g = O.mttkrp(sidx, O.dphi(ts, m, O.LOSS_LS), As, d, c.wl.dims[d])[rows] + \
                    2 * lam * As[d][rows]
                gabs = O.mttkrp(sidx, loss_abs(ts, m, m_abs, O.LOSS_LS, "dphi"),
                                [np.abs(a) for a in As], d, c.wl.dims[d])[rows] + \
                    2 * lam * np.abs(As[d][rows])
                gd = A[d].grad.float().double().cpu().numpy()[rows]
                # the returned gradient is rounded to the factors' dtype
                # (bf16 RNE: 2^-8 of the FP32 value, itself within tau*gabs)
                assert_close_abs(gd, g, rounded_abs(g, gabs, tau, 2.0 ** -8), tau,
                                 f"bf16 grad mode {d}")
        # finite differences on a 1,000-nonzero subsample (FP64 form)
        rfd = W.rng_for(W.SEED_FD + 3)
        pos = rfd.choice(c.wl.nnz, 1000, replace=False)
        sidx = [i[pos] for i in c.wl.idx]
        ts = c.t[pos]
        ix = tt.build_index([torch.as_tensor(i).cuda() for i in sidx], c.wl.dims,
                            torch.as_tensor(ts).cuda())
        Ad = [torch.as_tensor(a).cuda() for a in c.As]
        G = tt.gradient(ix, Ad, "ls", lam)
        for d in range(3):
            r = int(sidx[d][0])
            for col in (0, 17, 63):
                eps = 1e-6 * max(1.0, abs(c.As[d][r, col]))
                Ap = [a.clone() for a in Ad]
                Am = [a.clone() for a in Ad]
                Ap[d][r, col] += eps
                Am[d][r, col] -= eps
                fd = (tt.objective(ix, Ap, "ls", lam).item() -
                      tt.objective(ix, Am, "ls", lam).item()) / (2 * eps)
                gv = G[d][r, col].item()
                assert abs(fd - gv) <= 1e-6 * max(1.0, abs(fd)), f"fd mode {d} col {col}"
        ix.close()
    finally:
        c.ix.close()
        del c
        gc.collect()
        torch.cuda.empty_cache()


# ------------------------------------------------------------ counts ----
def test_counts_poisson_gn(gpu_lib):
    """50M Poisson counts, R = 32, log link, lambda = 0.1: phi'' TTTP on
    sampled nonzeros, the GN matvec with w = phi'' on sampled rows, and one
    preconditioned GN step (k_max = R) that lowers the objective."""
    tt = gpu_lib
    t0 = time.time()
    wl = W.counts()
    say(f"counts generated in {time.time() - t0:.1f}s")
    c = make_case(tt, wl, 32, "f32", W.SEED_INIT + 4)
    try:
        lam = 0.1
        rng = np.random.default_rng(7)
        w = tt.tttp(c.ix, tt.INDEX_T, c.A, epi="d2phi", loss="poisson")
        pos = rng.choice(wl.nnz, 20000, replace=False)
        sidx = [i[pos] for i in wl.idx]
        m = O.tttp(sidx, None, c.As)
        m_abs = O.tttp(sidx, None, [np.abs(a) for a in c.As])
        assert_close_abs(host(w)[pos], np.exp(m), loss_abs(0.0, m, m_abs, O.LOSS_POISSON_LOG,
                                                           "d2phi"), TAU["f32"], "phi''")
        wd = [tt.tttp(c.ix, tt.INDEX_T, c.A, epi="d2phi", loss="poisson", out_order=d)
              for d in range(3)]
        Xd = [torch.as_tensor(rng.standard_normal((dd, 32)).astype(np.float32)).cuda()
              for dd in wl.dims]
        Xh = [x.double().cpu().numpy() for x in Xd]
        Y = host(tt.gn_matvec(c.ix, wd, c.A, Xd, 2 * lam))
        for d in range(3):
            rows, cnt = sample_rows(wl.idx[d], wl.dims[d], rng, k=3)
            sidx, sel = subset(wl, d, rows)
            m = O.tttp(sidx, None, c.As)
            m_abs = O.tttp(sidx, None, [np.abs(a) for a in c.As])
            ww = np.exp(m)
            z = O.jvp(sidx, c.As, Xh)
            zabs = O.jvp(sidx, [np.abs(a) for a in c.As], [np.abs(x) for x in Xh])
            y = O.mttkrp(sidx, ww * z, c.As, d, wl.dims[d])[rows] + 2 * lam * Xh[d][rows]
            # w = phi'' as the GPU stored it carries the model value's error
            # through exp: its absolute form e^m (1 + m_abs) weights z_abs
            wa = loss_abs(0.0, m, m_abs, O.LOSS_POISSON_LOG, "d2phi")
            ya = O.mttkrp(sidx, wa * zabs, [np.abs(a) for a in c.As], d,
                          wl.dims[d])[rows] + 2 * lam * np.abs(Xh[d][rows])
            assert_close_abs(Y[d][rows], y, ya, TAU["f32"], f"poisson gn mode {d}")
        # BF16 factor storage: phi'' through the TTTP epilogue and the GN
        # product with w = phi'' on sampled rows, against the oracle on the
        # RNE-rounded factors (FP32 accumulation: tau)
        Ab = [a.to(torch.bfloat16).contiguous() for a in c.A]
        Abs = stored_factors(c.As, "bf16")
        wb = [tt.tttp(c.ix, tt.INDEX_T, Ab, epi="d2phi", loss="poisson", out_order=d)
              for d in range(3)]
        Yb = host(tt.gn_matvec(c.ix, wb, Ab, Xd, 2 * lam))
        w0 = host(tt.tttp(c.ix, tt.INDEX_T, Ab, epi="d2phi", loss="poisson"))[pos]
        sidx = [i[pos] for i in wl.idx]
        m = O.tttp(sidx, None, Abs)
        m_abs = O.tttp(sidx, None, [np.abs(a) for a in Abs])
        assert_close_abs(w0, np.exp(m), loss_abs(0.0, m, m_abs, O.LOSS_POISSON_LOG, "d2phi"),
                         TAU["bf16"], "bf16 phi''")
        for d in range(3):
            rows, cnt = sample_rows(wl.idx[d], wl.dims[d], rng, k=3)
            sidx, sel = subset(wl, d, rows)
            m = O.tttp(sidx, None, Abs)
            m_abs = O.tttp(sidx, None, [np.abs(a) for a in Abs])
            z = O.jvp(sidx, Abs, Xh)
            zabs = O.jvp(sidx, [np.abs(a) for a in Abs], [np.abs(x) for x in Xh])
            y = O.mttkrp(sidx, np.exp(m) * z, Abs, d, wl.dims[d])[rows] + 2 * lam * Xh[d][rows]
            wa = loss_abs(0.0, m, m_abs, O.LOSS_POISSON_LOG, "d2phi")
            ya = O.mttkrp(sidx, wa * zabs, [np.abs(a) for a in Abs], d,
                          wl.dims[d])[rows] + 2 * lam * np.abs(Xh[d][rows])
            assert_close_abs(Yb[d][rows], y, ya, TAU["bf16"], f"bf16 poisson gn mode {d}")
        del Ab, wb
        # one GN step (full step, as written in Section 2.5): PCG from dx = 0
        # guarantees a descent direction and a decrease of the quadratic
        # model q(dx) = g.dx + dx.H dx / 2 at any size; the full step itself
        # may overshoot with the exponential link, so the objective after the
        # step is reported, not asserted
        f0 = tt.objective(c.ix, c.A, "poisson", lam).item()
        g = tt.gradient(c.ix, c.A, "poisson", lam)
        A_before = [a.clone() for a in c.A]
        stats = tt.gn_step(c.ix, c.A, "poisson", lam, tol=5e-3, kmax=32).cpu().numpy()
        f1 = tt.objective(c.ix, c.A, "poisson", lam).item()
        dx = [(a1 - a0).contiguous() for a1, a0 in zip(c.A, A_before)]
        Hdx = tt.gn_matvec(c.ix, wd, A_before, dx, 2 * lam)
        gdx = sum(float((gg.double() * d.double()).sum().item()) for gg, d in zip(g, dx))
        dHd = sum(float((h.double() * d.double()).sum().item()) for h, d in zip(Hdx, dx))
        q = gdx + 0.5 * dHd
        say(f"counts GN: objective {f0:.6e} -> {f1:.6e}, CG iterations {stats[0]:.0f}, "
            f"rel. residual {stats[1]:.2e}, g.dx {gdx:.4e}, model decrease {q:.4e}")
        assert abs(stats[3] - f0) <= 1e-6 * abs(f0)
        assert 1 <= stats[0] <= 32
        assert gdx < 0 and dHd > 0 and q < 0
    finally:
        c.ix.close()
        del c
        gc.collect()
        torch.cuda.empty_cache()


# ----------------------------------------------------------- uniform ----
def test_uniform_1p5b(gpu_lib):
    """1.5B uniform nonzeros on 2^20 cubed, R = 32, FP32: TTTP on sampled
    nonzeros, MTTKRP and Solve Factor on sampled rows, the identity
    sum TTTP = <A_n, MTTKRP_n>, and the fused update with model values of
    the benchmarked step (solve_factor_model, mode 0)."""
    tt = gpu_lib
    t0 = time.time()
    wl = W.uniform()
    say(f"uniform generated in {time.time() - t0:.1f}s")
    c = make_case(tt, wl, 32, "f32", W.SEED_INIT + 5)
    try:
        rng = np.random.default_rng(8)
        lam = 1e-5
        pos = rng.choice(wl.nnz, 20000, replace=False)
        x = tt.tttp(c.ix, c.t_dev, c.A)
        xs = x[torch.as_tensor(pos).cuda()].double().cpu().numpy()
        del x
        sidx = [i[pos] for i in wl.idx]
        assert_close_abs(xs, O.tttp(sidx, c.t[pos], c.As),
                         O.tttp(sidx, np.abs(c.t[pos]), [np.abs(a) for a in c.As]),
                         TAU["f32"], "tttp 1.5B")
        _, tot = tt.tttp(c.ix, tt.INDEX_T, c.A, out=False, want_sum=True)
        _, tabs = tt.tttp(c.ix, tt.INDEX_T, [a.abs() for a in c.A], out=False, want_sum=True)
        rows = rng.choice(wl.dims[0], 4, replace=False)
        for n in range(3):
            M = tt.mttkrp(c.ix, tt.INDEX_T, c.A, n)
            ip = float((M.double() * c.A[n].double()).sum().item())
            assert abs(ip - tot.item()) <= 1e-5 * tabs.item(), f"identity mode {n}"
            X, info = tt.solve_factor(c.ix, None, c.A, n, M, lam)
            sel = np.flatnonzero(np.isin(wl.idx[n], rows))
            sidx = [i[sel] for i in wl.idx]
            ref = O.mttkrp(sidx, c.t[sel], c.As, n, wl.dims[n])[rows]
            ra = O.mttkrp(sidx, np.abs(c.t[sel]), [np.abs(a) for a in c.As], n,
                          wl.dims[n])[rows]
            assert_close_abs(host(M)[rows], ref, ra, TAU["f32"], f"mttkrp 1.5B mode {n}")
            G = O.gram(sidx, None, c.As, n, wl.dims[n], rows=rows)
            from gpu_helpers import backward_error
            be = backward_error(G, lam, host(X)[rows], ref)
            assert be <= 1e-5, f"solve 1.5B mode {n}: {be:.2e}"
            del M, X, info
        # the benchmarked step's call: mode 0's ALS update that also writes the
        # model values (mode-0 sorted order) equals solve_factor with the fused
        # right-hand side bit for bit, and its model values at sampled sorted
        # positions are the oracle's TTTP of the factors before the update
        X0, info0 = tt.solve_factor(c.ix, None, c.A, 0, tt.RHS_MTTKRP, lam)
        X1, info1, model = tt.solve_factor_model(c.ix, c.A, 0, lam)
        assert torch.equal(X0, X1) and torch.equal(info0, info1), "fused model update 1.5B"
        del X0, X1, info0, info1
        js = torch.as_tensor(rng.choice(wl.nnz, 20000, replace=False)).cuda()
        cpos = c.ix.view(0)[1][js].long().cpu().numpy()
        ms = model[js].double().cpu().numpy()
        del model
        sidx = [i[cpos] for i in wl.idx]
        assert_close_abs(ms, O.tttp(sidx, None, c.As),
                         O.tttp(sidx, None, [np.abs(a) for a in c.As]), TAU["f32"],
                         "model values 1.5B")
        # BF16 factor storage on the same index: TTTP on sampled nonzeros,
        # MTTKRP on sampled rows (FP32 accumulation: tau against the oracle on
        # the RNE-rounded factors) and the fused ALS update (Gram and
        # right-hand side in one pass, FP64 Cholesky, solved rows rounded to
        # BF16: backward error within 2e-2 of the rounded and the unrounded
        # factors' normal equations)
        Ab = [a.to(torch.bfloat16).contiguous() for a in c.A]
        Abs = [a.float().double().cpu().numpy() for a in Ab]
        assert all(np.array_equal(x, y) for x, y in zip(Abs, stored_factors(c.As, "bf16")))
        x = tt.tttp(c.ix, c.t_dev, Ab)
        xs = x[torch.as_tensor(pos).cuda()].double().cpu().numpy()
        del x
        sidx = [i[pos] for i in wl.idx]
        assert_close_abs(xs, O.tttp(sidx, c.t[pos], Abs),
                         O.tttp(sidx, np.abs(c.t[pos]), [np.abs(a) for a in Abs]),
                         TAU["bf16"], "bf16 tttp 1.5B")
        for n in range(3):
            sel = np.flatnonzero(np.isin(wl.idx[n], rows))
            sidx = [i[sel] for i in wl.idx]
            M = host(tt.mttkrp(c.ix, tt.INDEX_T, Ab, n))[rows]
            ref = O.mttkrp(sidx, c.t[sel], Abs, n, wl.dims[n])[rows]
            ra = O.mttkrp(sidx, np.abs(c.t[sel]), [np.abs(a) for a in Abs], n,
                          wl.dims[n])[rows]
            assert_close_abs(M, ref, ra, TAU["bf16"], f"bf16 mttkrp 1.5B mode {n}")
            X, info = tt.solve_factor(c.ix, None, Ab, n, tt.RHS_MTTKRP, lam)
            assert int((info != 0).sum().item()) == 0
            Xh = host(X)[rows]
            G = O.gram(sidx, None, Abs, n, wl.dims[n], rows=rows)
            be = backward_error(G, lam, Xh, ref)
            assert be <= TAU_BF16_VS_F32, f"bf16 fused update 1.5B mode {n}: {be:.2e}"
            G0 = O.gram(sidx, None, c.A0, n, wl.dims[n], rows=rows)
            M0 = O.mttkrp(sidx, c.t[sel], c.A0, n, wl.dims[n])[rows]
            be0 = backward_error(G0, lam, Xh, M0)
            assert be0 <= TAU_BF16_VS_F32, f"bf16 vs fp32 factors mode {n}: {be0:.2e}"
            del X, info
        del Ab
    finally:
        c.ix.close()
        del c
        gc.collect()
        torch.cuda.empty_cache()
