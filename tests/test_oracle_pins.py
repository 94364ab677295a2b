"""Pins of the FP64 oracle against brute force, closed forms, invariants and
library routines (CPU only).  Each check is chosen so that a plausible slip
in the oracle (a dropped term, a wrong index, a transposed operand, a missing
weight) fails it."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1910_02371_amd import workloads as W


def small(dims, m, seed, rank=3, R=None):
    wl = W.random_tensor(dims, m, seed, rank=rank)
    rng = np.random.default_rng(seed + 7)
    R = R or rank + 1
    A = [rng.standard_normal((I, R)) for I in dims]
    return wl, A


def dense_cp(A, dims, skip=()):
    """Dense CP tensor by explicit loops over every entry and every r."""
    R = A[next(n for n in range(len(dims)) if n not in skip)].shape[1]
    T = np.zeros(dims)
    for ii in itertools.product(*[range(d) for d in dims]):
        v = 0.0
        for r in range(R):
            p = 1.0
            for n, i in enumerate(ii):
                if n in skip:
                    continue
                p *= A[n][i, r]
            v += p
        T[ii] = v
    return T


# ---------------------------------------------------------------- index ----
@pytest.mark.parametrize("case", ["random", "sorted", "reverse", "one_row",
                                  "empty_rows", "single"])
def test_index_brute_force(case):
    rng = np.random.default_rng(3)
    dims = (7, 5, 6)
    if case == "single":
        idx = [np.array([3]), np.array([1]), np.array([5])]
    else:
        m = 60
        idx = [rng.integers(0, d, m) for d in dims]
        if case == "sorted":
            o = np.lexsort((idx[2], idx[1], idx[0]))
            idx = [a[o] for a in idx]
        elif case == "reverse":
            o = np.lexsort((idx[2], idx[1], idx[0]))[::-1]
            idx = [a[o] for a in idx]
        elif case == "one_row":
            idx[1][:] = 2
        elif case == "empty_rows":
            idx[0] = np.where(idx[0] % 2 == 0, idx[0], 0)
    ix = O.build_index(idx, dims)
    m = len(idx[0])
    for n in range(3):
        d = ix[n]
        # brute-force stable sort: walk keys in increasing order, COO order
        # inside each key
        expect = [e for k in range(dims[n]) for e in range(m) if idx[n][e] == k]
        assert d["perm"].tolist() == expect
        cnt = [sum(1 for e in range(m) if idx[n][e] == k) for k in range(dims[n])]
        assert d["cnt"].tolist() == cnt
        assert d["ptr"].tolist() == [sum(cnt[:k]) for k in range(dims[n] + 1)]
        assert d["rows"].tolist() == [k for k in range(dims[n]) if cnt[k] > 0]
        for p in range(3):
            if p != n:
                assert d["other"][p].tolist() == [idx[p][e] for e in expect]


# ----------------------------------------------------------------- TTTP ----
@pytest.mark.parametrize("dims,skip", [((4, 3, 5), ()), ((4, 3, 5), (1,)),
                                       ((3, 4, 2, 3), ()), ((3, 4, 2, 3), (1, 3))])
def test_tttp_dense_masked(dims, skip):
    rng = np.random.default_rng(11)
    R = 3
    A = [rng.standard_normal((d, R)) for d in dims]
    T = dense_cp(A, dims, skip)
    m = 17
    keys = rng.choice(int(np.prod(dims)), m, replace=False)
    idx = list(np.unravel_index(keys, dims))
    s = rng.standard_normal(m)
    Ain = [None if n in skip else A[n] for n in range(len(dims))]
    x = O.tttp(idx, s, Ain)
    np.testing.assert_allclose(x, s * T[tuple(idx)], rtol=1e-13, atol=1e-13)


def test_tttp_sddmm():
    rng = np.random.default_rng(5)
    U, V = rng.standard_normal((6, 4)), rng.standard_normal((7, 4))
    S = rng.standard_normal((6, 7)) * (rng.random((6, 7)) < 0.4)
    i, j = np.nonzero(S)
    x = O.tttp([i, j], S[i, j], [U, V])
    np.testing.assert_allclose(x, (S * (U @ V.T))[i, j], rtol=1e-13)


def test_tttp_ones_and_vectors():
    wl, _ = small((5, 6, 7), 30, 1)
    ones = [np.ones((d, 4)) for d in wl.dims]
    np.testing.assert_allclose(O.tttp(wl.idx, wl.t, ones), 4 * wl.t)
    vec = [np.arange(1, d + 1, dtype=float) for d in wl.dims]
    expect = wl.t * np.prod([vec[n][wl.idx[n]] for n in range(3)], axis=0)
    np.testing.assert_allclose(O.tttp(wl.idx, wl.t, vec), expect)


def test_tttp_hand_example():
    # 2x2x2 with rank 2, integers: m_(1,0,1) = 1*3*5 + 2*4*6 = 63
    U = np.array([[9., 9.], [1., 2.]])
    V = np.array([[3., 4.], [9., 9.]])
    Wm = np.array([[9., 9.], [5., 6.]])
    x = O.tttp([np.array([1]), np.array([0]), np.array([1])], np.array([2.0]),
               [U, V, Wm])
    assert x.tolist() == [126.0]


# --------------------------------------------------------------- MTTKRP ----
@pytest.mark.parametrize("n", [0, 1, 2])
def test_mttkrp_khatri_rao(n):
    rng = np.random.default_rng(21 + n)
    dims = (4, 5, 3)
    R = 3
    A = [rng.standard_normal((d, R)) for d in dims]
    m = 25
    keys = rng.choice(int(np.prod(dims)), m, replace=False)
    idx = list(np.unravel_index(keys, dims))
    s = rng.standard_normal(m)
    S = np.zeros(dims)
    S[tuple(idx)] = s
    others = [p for p in range(3) if p != n]
    # mode-n unfolding: columns enumerate (i_p, i_q) with the later mode fastest
    Xn = np.moveaxis(S, n, 0).reshape(dims[n], -1)
    KR = np.zeros((dims[others[0]] * dims[others[1]], R))
    for a in range(dims[others[0]]):
        for b in range(dims[others[1]]):
            KR[a * dims[others[1]] + b] = A[others[0]][a] * A[others[1]][b]
    np.testing.assert_allclose(O.mttkrp(idx, s, A, n, dims[n]), Xn @ KR,
                               rtol=1e-12, atol=1e-12)


def test_tttp_mttkrp_cross_identity():
    wl, A = small((9, 8, 7), 120, 4, R=5)
    x = O.tttp(wl.idx, wl.t, A)
    for n in range(3):
        Y = O.mttkrp(wl.idx, wl.t, A, n, wl.dims[n])
        assert np.isclose(x.sum(), np.sum(A[n] * Y), rtol=1e-12)


# ----------------------------------------------------------------- Gram ----
def test_gram_explicit_and_quadratic_identity():
    wl, A = small((6, 7, 5), 80, 8, R=4)
    rng = np.random.default_rng(2)
    w = rng.random(wl.nnz) + 0.1
    for n in range(3):
        G = O.gram(wl.idx, w, A, n, wl.dims[n])
        for i in range(wl.dims[n]):
            Gi = np.zeros((4, 4))
            for e in range(wl.nnz):
                if wl.idx[n][e] != i:
                    continue
                h = np.ones(4)
                for p in range(3):
                    if p != n:
                        h = h * A[p][wl.idx[p][e]]
                Gi += w[e] * np.outer(h, h)
            np.testing.assert_allclose(G[i], Gi, rtol=1e-12, atol=1e-12)
        mvals = O.tttp(wl.idx, None, A)
        quad = np.einsum("ir,irs,is->", A[n], G, A[n])
        assert np.isclose(quad, np.sum(w * mvals ** 2), rtol=1e-11)


def test_gram_full_tensor_hadamard_of_grams():
    # Omega = all entries: G^(i) = (V^T V) * (W^T W) for every i (the CP-ALS
    # normal equations of plain decomposition, Appendix A).
    dims = (3, 4, 5)
    rng = np.random.default_rng(9)
    A = [rng.standard_normal((d, 3)) for d in dims]
    idx = [a.ravel() for a in np.meshgrid(*[np.arange(d) for d in dims],
                                          indexing="ij")]
    for n in range(3):
        o = [p for p in range(3) if p != n]
        H = (A[o[0]].T @ A[o[0]]) * (A[o[1]].T @ A[o[1]])
        G = O.gram(idx, None, A, n, dims[n])
        for i in range(dims[n]):
            np.testing.assert_allclose(G[i], H, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- solve ----
def test_solve_ridge_lstsq_and_backward_error():
    wl, A = small((6, 5, 7), 90, 12, R=4)
    lam = 0.3
    for n in range(3):
        M = O.mttkrp(wl.idx, wl.t, A, n, wl.dims[n])
        X, info = O.solve_factor(wl.idx, None, A, n, wl.dims[n], M, lam)
        assert (info == 0).all()
        ix = O.build_index(wl.idx, wl.dims)[n]
        G = O.gram(wl.idx, None, A, n, wl.dims[n])
        for i in range(wl.dims[n]):
            H, sel = O.row_design(wl.idx, A, n, ix, i)
            lhs = np.vstack([H, np.sqrt(lam) * np.eye(4)])
            rhs = np.concatenate([wl.t[sel], np.zeros(4)])
            ref = np.linalg.lstsq(lhs, rhs, rcond=None)[0]
            np.testing.assert_allclose(X[i], ref, rtol=1e-9, atol=1e-11)
            S = G[i] + lam * np.eye(4)
            be = np.linalg.norm(S @ X[i] - M[i]) / (
                np.linalg.norm(S, 2) * np.linalg.norm(X[i]) + np.linalg.norm(M[i]))
            assert be < 1e-14


def test_solve_rank1_is_ccd_update():
    # R = 1: u_i = sum v w t / (lam + sum v^2 w^2) (Section 2.3)
    wl, _ = small((5, 6, 4), 50, 13)
    rng = np.random.default_rng(1)
    A = [rng.standard_normal((d, 1)) for d in wl.dims]
    lam = 0.2
    M = O.mttkrp(wl.idx, wl.t, A, 0, 5)
    X, _ = O.solve_factor(wl.idx, None, A, 0, 5, M, lam)
    for i in range(5):
        num = den = 0.0
        for e in range(wl.nnz):
            if wl.idx[0][e] == i:
                v, w_ = A[1][wl.idx[1][e], 0], A[2][wl.idx[2][e], 0]
                num += v * w_ * wl.t[e]
                den += v * v * w_ * w_
        assert np.isclose(X[i, 0], num / (lam + den), rtol=1e-12)


def test_solve_info_conventions():
    G = np.zeros((3, 2, 2))
    G[1] = np.array([[1.0, 0.0], [0.0, -2.0]])     # indefinite: minor 2 fails
    G[2] = np.array([[4.0, 2.0], [2.0, 5.0]])
    M = np.ones((3, 2))
    X, info = O.solve_rows(G, M, 0.0)
    assert info.tolist() == [1, 2, 0]
    assert (X[0] == 0).all() and (X[1] == 0).all()
    np.testing.assert_allclose(G[2] @ X[2], M[2])
    # empty row with lam > 0: x = M / lam
    X, info = O.solve_rows(np.zeros((1, 2, 2)), np.array([[2.0, 4.0]]), 0.5)
    assert info.tolist() == [0]
    np.testing.assert_allclose(X, [[4.0, 8.0]], rtol=1e-15)


def test_cholesky_info_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(20):
        B = rng.standard_normal((5, 5))
        S = B @ B.T - rng.random() * 6 * np.eye(5)
        k = O.cholesky_info(S)
        minors = [np.linalg.det(S[:j, :j]) > 0 for j in range(1, 6)]
        expect = 0 if all(minors) else minors.index(False) + 1
        assert k == expect


# ----------------------------------------------------------------- loss ----
@pytest.mark.parametrize("loss", [O.LOSS_LS, O.LOSS_POISSON_LOG])
def test_loss_derivatives_fd(loss):
    t = np.array([0.0, 1.0, 3.0, 5.0])
    m = np.array([-0.7, 0.2, 1.1, 1.9])
    h = 1e-5
    fd1 = (O.phi(t, m + h, loss) - O.phi(t, m - h, loss)) / (2 * h)
    fd2 = (O.dphi(t, m + h, loss) - O.dphi(t, m - h, loss)) / (2 * h)
    np.testing.assert_allclose(O.dphi(t, m, loss), fd1, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(O.d2phi(t, m, loss), fd2, rtol=1e-7, atol=1e-9)
    if loss == O.LOSS_LS:
        assert O.phi(3.0, 1.0, loss) == 4.0
    else:
        assert np.isclose(O.phi(2.0, 0.0, loss), 1.0)


# ------------------------------------------------------------- gradient ----
@pytest.mark.parametrize("loss", [O.LOSS_LS, O.LOSS_POISSON_LOG])
def test_gradient_central_fd(loss):
    wl, A = small((4, 5, 3), 30, 17, R=3)
    A = [0.5 * a for a in A]
    t = np.abs(np.round(wl.t)) if loss == O.LOSS_POISSON_LOG else wl.t
    lam = 0.05
    g = O.gradient(wl.idx, t, A, loss, lam, wl.dims)
    for d in range(3):
        for i in range(wl.dims[d]):
            for r in range(3):
                eps = 1e-6 * max(1.0, abs(A[d][i, r]))
                Ap = [a.copy() for a in A]
                Am = [a.copy() for a in A]
                Ap[d][i, r] += eps
                Am[d][i, r] -= eps
                fd = (O.objective(wl.idx, t, Ap, loss, lam) -
                      O.objective(wl.idx, t, Am, loss, lam)) / (2 * eps)
                assert abs(fd - g[d][i, r]) <= 1e-6 * max(1.0, abs(fd))


# ------------------------------------------------------------ GN matvec ----
def jacobian(idx, A, dims):
    """Explicit J: dm_e / dA_p[i, r] = [i_p(e) == i] prod_{q != p} A_q[i_q(e), r]."""
    m = len(idx[0])
    R = A[0].shape[1]
    offs = np.concatenate([[0], np.cumsum([d * R for d in dims])])
    J = np.zeros((m, offs[-1]))
    for e in range(m):
        for p in range(len(dims)):
            for r in range(R):
                v = 1.0
                for q in range(len(dims)):
                    if q != p:
                        v *= A[q][idx[q][e], r]
                J[e, offs[p] + idx[p][e] * R + r] += v
    return J


def test_gn_matvec_explicit_jacobian_symmetry_psd():
    wl, A = small((4, 3, 5), 25, 31, R=2)
    rng = np.random.default_rng(6)
    w = rng.random(wl.nnz) + 0.5
    lam2 = 0.3
    J = jacobian(wl.idx, A, wl.dims)
    Hm = J.T @ (w[:, None] * J) + lam2 * np.eye(J.shape[1])
    X = [rng.standard_normal(a.shape) for a in A]
    Y = O.gn_matvec(wl.idx, w, A, X, lam2, wl.dims)
    np.testing.assert_allclose(np.concatenate([y.ravel() for y in Y]),
                               Hm @ np.concatenate([x.ravel() for x in X]),
                               rtol=1e-11, atol=1e-11)
    X2 = [rng.standard_normal(a.shape) for a in A]
    Y2 = O.gn_matvec(wl.idx, w, A, X2, lam2, wl.dims)
    lhs = sum(np.sum(y * x2) for y, x2 in zip(Y, X2))
    rhs = sum(np.sum(x * y2) for x, y2 in zip(X, Y2))
    assert np.isclose(lhs, rhs, rtol=1e-11)
    assert np.linalg.eigvalsh(Hm).min() > 0
    # block (d, d) of the operator is the Solve Factor Gram on x_d
    for d in range(3):
        Xd = [np.zeros_like(a) for a in A]
        Xd[d] = X[d]
        Yd = O.gn_matvec(wl.idx, w, A, Xd, 0.0, wl.dims)[d]
        G = O.gram(wl.idx, w, A, d, wl.dims[d])
        np.testing.assert_allclose(Yd, np.einsum("irs,is->ir", G, X[d]),
                                   rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("loss", [O.LOSS_LS, O.LOSS_POISSON_LOG])
def test_newton_matvec_is_gradient_derivative(loss):
    """The full Hessian-vector product equals the central difference of the
    gradient in the direction X (error O(eps^2)); the GN operator differs
    from it by the phi' terms, so it must not match."""
    wl = W.random_tensor((6, 5, 7), 80, 13, rank=2)
    rng = np.random.default_rng(4)
    A = [0.5 * rng.standard_normal((d, 3)) for d in wl.dims]
    X = [rng.standard_normal((d, 3)) for d in wl.dims]
    t = wl.t if loss == O.LOSS_LS else np.round(np.exp(wl.t))
    lam, eps = 0.05, 1e-5
    gp = O.gradient(wl.idx, t, [a + eps * x for a, x in zip(A, X)], loss, lam, wl.dims)
    gm = O.gradient(wl.idx, t, [a - eps * x for a, x in zip(A, X)], loss, lam, wl.dims)
    fd = [(p - q) / (2 * eps) for p, q in zip(gp, gm)]
    Y = O.newton_matvec(wl.idx, t, A, X, 2 * lam, wl.dims, loss)
    scale = max(np.abs(f).max() for f in fd)
    for d in range(3):
        np.testing.assert_allclose(Y[d], fd[d], rtol=0, atol=1e-7 * scale)
    m = O.tttp(wl.idx, None, A)
    G = O.gn_matvec(wl.idx, O.d2phi(t, m, loss), A, X, 2 * lam, wl.dims)
    assert max(np.abs(g - f).max() for g, f in zip(G, fd)) > 1e-3 * scale


def test_newton_matvec_symmetric_and_gn_at_zero_residual():
    wl = W.random_tensor((6, 5, 7), 80, 17, rank=2)
    rng = np.random.default_rng(5)
    A = [rng.standard_normal((d, 3)) for d in wl.dims]
    X1 = [rng.standard_normal((d, 3)) for d in wl.dims]
    X2 = [rng.standard_normal((d, 3)) for d in wl.dims]
    t = np.round(np.exp(0.3 * wl.t))
    L = O.LOSS_POISSON_LOG
    Y1 = O.newton_matvec(wl.idx, t, A, X1, 0.2, wl.dims, L)
    Y2 = O.newton_matvec(wl.idx, t, A, X2, 0.2, wl.dims, L)
    a = sum(np.sum(y * x) for y, x in zip(Y1, X2))
    b = sum(np.sum(y * x) for y, x in zip(Y2, X1))
    assert np.isclose(a, b, rtol=1e-11)
    # least squares with t equal to the model: phi' = 0, so Newton = GN
    tm = O.tttp(wl.idx, None, A)
    Yn = O.newton_matvec(wl.idx, tm, A, X1, 0.2, wl.dims, O.LOSS_LS)
    Yg = O.gn_matvec(wl.idx, np.full(len(tm), 2.0), A, X1, 0.2, wl.dims)
    for d in range(3):
        np.testing.assert_allclose(Yn[d], Yg[d], rtol=1e-12, atol=1e-12)


def test_jvp_matches_fd_of_model():
    wl, A = small((4, 5, 3), 20, 41, R=3)
    rng = np.random.default_rng(8)
    X = [rng.standard_normal(a.shape) for a in A]
    h = 1e-6
    mp = O.tttp(wl.idx, None, [a + h * x for a, x in zip(A, X)])
    mm = O.tttp(wl.idx, None, [a - h * x for a, x in zip(A, X)])
    np.testing.assert_allclose(O.jvp(wl.idx, A, X), (mp - mm) / (2 * h),
                               rtol=1e-7, atol=1e-8)


# ------------------------------------------------------------------ PCG ----
def test_pcg_small_spd():
    rng = np.random.default_rng(12)
    n = 12
    B = rng.standard_normal((n, n))
    S = B @ B.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)
    x, k, rel = O.pcg(lambda X: [S @ X[0]], lambda X: [X[0].copy()], [b], 1e-12, n + 5)
    np.testing.assert_allclose(x[0], np.linalg.solve(S, b), rtol=1e-8, atol=1e-10)
    assert k <= n + 1
    # exact inverse as preconditioner: one iteration
    Si = np.linalg.inv(S)
    x, k, rel = O.pcg(lambda X: [S @ X[0]], lambda X: [Si @ X[0]], [b], 1e-10, 5)
    assert k == 1
    np.testing.assert_allclose(x[0], np.linalg.solve(S, b), rtol=1e-9)


def test_gn_step_decreases_objective():
    # random planted tensor, 30% observed (shape of the dense GN experiment)
    wl = W.random_tensor((8, 8, 8), 154, 77, rank=3, noise=0.0)
    A = W.init_factors(wl.dims, 3, np.mean(wl.t), 5, dtype=np.float64)
    lam = 1e-3
    f0 = O.objective(wl.idx, wl.t, A, O.LOSS_LS, lam)
    A1, it, rel = O.gn_step(wl.idx, wl.t, A, wl.dims, O.LOSS_LS, lam, 5e-3, 30)
    assert O.objective(wl.idx, wl.t, A1, O.LOSS_LS, lam) < f0
    assert it >= 1


def _gn_problem(loss, seed):
    """A tiny tensor for the Gauss-Newton composition pins: least squares
    with planted values, or Poisson counts drawn at a planted log rate."""
    wl = W.random_tensor((4, 5, 3), 26, seed, rank=2, noise=0.05)
    rng = np.random.default_rng(seed + 1)
    A = [0.7 * rng.random((I, 2)) + 0.2 for I in wl.dims]
    t = np.asarray(wl.t, dtype=np.float64)
    if loss == O.LOSS_POISSON_LOG:
        t = rng.poisson(np.exp(0.5 * t)).astype(np.float64)
    return wl, t, A


def _gn_explicit(wl, t, A, loss, lam):
    """H = J^T diag(phi'') J + 2 lam I, the gradient J^T phi' + 2 lam vec(A)
    and the block-diagonal preconditioner (each mode's diagonal block of H),
    all from the explicit Jacobian and the closed-form loss derivatives."""
    J = jacobian(wl.idx, A, wl.dims)
    a = np.concatenate([x.ravel() for x in A])
    m = J.shape[0]
    # model values from the Jacobian: each nonzero's row of J dotted with the
    # factors counts every rank-1 term N times (once per mode)
    mv = (J @ a) / len(A)
    if loss == O.LOSS_LS:
        d1, d2 = 2.0 * (mv - t), np.full(m, 2.0)
    else:
        d1, d2 = np.exp(mv) - t, np.exp(mv)
    n = J.shape[1]
    H = J.T @ (d2[:, None] * J) + 2.0 * lam * np.eye(n)
    g = J.T @ d1 + 2.0 * lam * a
    P = np.zeros_like(H)
    off = 0
    for I in wl.dims:
        sl = slice(off, off + I * A[0].shape[1])
        P[sl, sl] = H[sl, sl]
        off += I * A[0].shape[1]
    return H, g, P


def _step(A1, A):
    return np.concatenate([(x1 - x).ravel() for x1, x in zip(A1, A)])


@pytest.mark.parametrize("loss", [O.LOSS_LS, O.LOSS_POISSON_LOG])
def test_gn_step_converged_is_newton_system_solution(loss):
    """Section 2.5: with a tight tolerance and enough iterations the step is
    -(J^T diag(phi'') J + 2 lam I)^{-1} grad f, the full Gauss-Newton step
    (fails for lam instead of 2 lam in the operator, or for 2 instead of
    phi'' as the operator weights)."""
    lam = 0.05
    wl, t, A = _gn_problem(loss, 91)
    H, g, _ = _gn_explicit(wl, t, A, loss, lam)
    A1, it, rel = O.gn_step(wl.idx, t, A, wl.dims, loss, lam, 1e-14, 4 * H.shape[0])
    np.testing.assert_allclose(_step(A1, A), -np.linalg.solve(H, g), rtol=1e-8, atol=1e-10)
    assert rel <= 1e-14


@pytest.mark.parametrize("loss", [O.LOSS_LS, O.LOSS_POISSON_LOG])
def test_gn_step_one_iteration_is_preconditioned_steepest_descent(loss):
    """One PCG iteration from x0 = 0 gives alpha P^{-1} r0 with r0 = -grad f,
    P the block diagonal of J^T diag(phi'') J + 2 lam I and
    alpha = (r0 . P^{-1} r0) / (z0 . H z0): pins the preconditioner's weights
    (phi'') and shift (2 lam) separately from the operator's."""
    lam = 0.05
    wl, t, A = _gn_problem(loss, 92)
    H, g, P = _gn_explicit(wl, t, A, loss, lam)
    r0 = -g
    z0 = np.linalg.solve(P, r0)
    alpha = (r0 @ z0) / (z0 @ H @ z0)
    A1, it, _ = O.gn_step(wl.idx, t, A, wl.dims, loss, lam, 0.0, 1)
    assert it == 1
    np.testing.assert_allclose(_step(A1, A), alpha * z0, rtol=1e-10, atol=1e-12)


def test_gn_step_stops_on_unpreconditioned_residual():
    """The PCG stop rule (Sections 5.6/5.7) compares the unpreconditioned
    residual norm ||b - H x_k|| / ||b|| with the tolerance.  A tolerance is
    chosen at which that norm and the preconditioned one sqrt(r.P^{-1}r)
    (relative to its initial value) first fall below it at different
    iterations; the step must stop at the unpreconditioned crossing and
    equal that iterate."""
    lam = 0.05
    loss = O.LOSS_POISSON_LOG
    wl, t, A = _gn_problem(loss, 93)
    H, g, P = _gn_explicit(wl, t, A, loss, lam)
    b = -g
    Pi = np.linalg.inv(P)
    xs, un, pre = [], [], []
    for k in range(1, 12):
        A1, it, _ = O.gn_step(wl.idx, t, A, wl.dims, loss, lam, 0.0, k)
        assert it == k
        x = _step(A1, A)
        r = b - H @ x
        xs.append(x)
        un.append(np.linalg.norm(r) / np.linalg.norm(b))
        pre.append(np.sqrt(r @ Pi @ r) / np.sqrt(b @ Pi @ b))

    def first(seq, tol):
        return next((k + 1 for k, v in enumerate(seq) if v <= tol), None)

    tol = None
    for cand in np.geomspace(0.5, 1e-6, 200):
        ku, kp = first(un, cand), first(pre, cand)
        if ku is not None and kp is not None and ku != kp:
            tol = float(cand)
            break
    assert tol is not None, "no tolerance separates the two residual measures"
    ku = first(un, tol)
    A1, it, rel = O.gn_step(wl.idx, t, A, wl.dims, loss, lam, tol, 50)
    assert it == ku and it != first(pre, tol)
    np.testing.assert_allclose(_step(A1, A), xs[ku - 1], rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------ ALS ----
def test_als_monotone_gradient_and_fast_loss():
    wl = W.random_tensor((9, 10, 8), 200, 55, rank=3)
    lam = 1e-3
    A = W.init_factors(wl.dims, 4, float(np.mean(wl.t)), 3, dtype=np.float64)
    f_prev = O.objective(wl.idx, wl.t, A, O.LOSS_LS, lam)
    for sweep in range(3):
        for n in range(3):
            M = O.mttkrp(wl.idx, wl.t, A, n, wl.dims[n])
            G = O.gram(wl.idx, None, A, n, wl.dims[n])
            X, info = O.solve_rows(G, M, lam)
            A = list(A)
            A[n] = X
            f = O.objective(wl.idx, wl.t, A, O.LOSS_LS, lam)
            assert f <= f_prev * (1 + 1e-12)
            f_prev = f
            # gradient of f = sum (t-m)^2 + lam sum ||A||^2 with respect to
            # the solved mode vanishes: 2 (G x - M) + 2 lam x = 0 (Table 1;
            # the factor 2 cancels in the Section 2.2 normal equations)
            g = O.gradient(wl.idx, wl.t, A, O.LOSS_LS, lam, wl.dims)[n]
            assert np.abs(g).max() < 1e-9 * max(1.0, np.abs(M).max())
            mvals = O.tttp(wl.idx, None, A)
            ls = np.sum((wl.t - mvals) ** 2)
            assert np.isclose(O.als_fast_loss(wl.t, A[n], G, M), ls, rtol=1e-9)


@pytest.mark.slow
def test_als_cube_converges_to_noise_floor():
    wl = W.cube()
    A = W.init_factors(wl.dims, 10, float(np.mean(wl.t)), W.SEED_INIT + 1,
                       dtype=np.float64)
    r = []
    for _ in range(30):
        A, _ = O.als_sweep(wl.idx, wl.t, A, wl.dims, 1e-5)
        r.append(O.rmse(wl.idx, wl.t, A))
    assert all(b <= a * (1 + 1e-9) for a, b in zip(r, r[1:]))
    # a least-squares fit with dof = 3 * 200 * 10 free parameters to m noisy
    # observations (sigma = 0.01) leaves a training residual of about
    # sigma * sqrt(1 - dof / m) = 0.00922 once converged
    floor = 0.01 * np.sqrt(1.0 - 3 * 200 * 10 / wl.nnz)
    assert abs(r[-1] - floor) <= 0.05 * floor, (r[-1], floor)


# ------------------------------------------------------------------ GAM ----
def test_gam_least_squares_is_als():
    """Least squares: the row subproblem is quadratic, so one Newton step
    from any start lands on its minimizer, the ALS solve (Section 2.2).  The
    GAM sweep (gradient, phi'' Gram, shift 2 lam) must equal the ALS sweep
    (MTTKRP of t, Omega-hat Gram, shift lam) from a random start, and a
    second inner iteration must not move it."""
    wl = W.random_tensor((9, 10, 8), 200, 55, rank=3)
    lam = 1e-3
    A = W.init_factors(wl.dims, 4, float(np.mean(wl.t)), 3, dtype=np.float64)
    Aa, _ = O.als_sweep(wl.idx, wl.t, A, wl.dims, lam)
    Ag, counts, infos = O.gam_sweep(wl.idx, wl.t, A, wl.dims, O.LOSS_LS, lam, 0.0, 1)
    assert counts == [1, 1, 1] and all((i == 0).all() for i in infos)
    for d in range(3):
        np.testing.assert_allclose(Ag[d], Aa[d], rtol=1e-9, atol=1e-12)
    # the stop rule: the second Newton step of each mode is ~0
    Ag2, counts2, _ = O.gam_sweep(wl.idx, wl.t, A, wl.dims, O.LOSS_LS, lam, 1e-6, 5)
    assert counts2 == [2, 2, 2]
    for d in range(3):
        np.testing.assert_allclose(Ag2[d], Aa[d], rtol=1e-8, atol=1e-11)


def test_gam_poisson_rows_minimize_their_objective():
    """Poisson log link: after converged inner iterations on mode 0, every
    row of A_0 minimizes its own objective
        sum_{e in row i} [exp(m_e) - t_e m_e] + lam ||u_i||^2,
    found here by scipy's BFGS from the loss phi alone (no phi' or phi'' of
    the oracle), and the objective does not increase mode by mode."""
    import scipy.optimize
    wl = W.random_tensor((7, 6, 5), 90, 31, rank=2, noise=0.0)
    t = np.round(np.exp(0.5 * wl.t))
    lam = 0.1
    A = W.init_factors(wl.dims, 3, float(np.log(np.mean(t) + 1)), 4, dtype=np.float64)
    f_prev = O.objective(wl.idx, t, A, O.LOSS_POISSON_LOG, lam)
    A1, counts, _ = O.gam_sweep(wl.idx, t, A, wl.dims, O.LOSS_POISSON_LOG, lam, 0.0, 25)
    # mode 0 was solved first, with A[1], A[2] still the initial factors
    B = [A1[0], A[1], A[2]]
    idx = [np.asarray(a) for a in wl.idx]
    for i in range(wl.dims[0]):
        sel = np.nonzero(idx[0] == i)[0]
        H = A[1][idx[1][sel]] * A[2][idx[2][sel]]

        def f(u):
            mv = H @ u
            return float(np.sum(O.phi(t[sel], mv, O.LOSS_POISSON_LOG)) + lam * u @ u)

        res = scipy.optimize.minimize(f, np.zeros(3), method="BFGS",
                                      options=dict(gtol=1e-11, maxiter=2000))
        np.testing.assert_allclose(B[0][i], res.x, rtol=1e-5, atol=1e-6)
        assert f(B[0][i]) <= res.fun + 1e-9 * abs(res.fun)
    # block minimization: the objective after the sweep is below the start
    assert O.objective(wl.idx, t, A1, O.LOSS_POISSON_LOG, lam) < f_prev


def test_gam_stop_rule():
    """tol > 0 stops a mode at the first iteration whose step is at most
    tol times the updated factor's norm; tol = 0 runs max_inner."""
    wl = W.random_tensor((7, 6, 5), 90, 31, rank=2, noise=0.0)
    t = np.round(np.exp(0.5 * wl.t))
    A = W.init_factors(wl.dims, 3, float(np.log(np.mean(t) + 1)), 4, dtype=np.float64)
    _, c0, _ = O.gam_sweep(wl.idx, t, A, wl.dims, O.LOSS_POISSON_LOG, 0.1, 0.0, 4)
    assert c0 == [4, 4, 4]
    _, c1, _ = O.gam_sweep(wl.idx, t, A, wl.dims, O.LOSS_POISSON_LOG, 0.1, 1e-3, 25)
    assert all(1 <= c < 25 for c in c1)
    # replay mode 0 by hand to check the count
    An = [a.copy() for a in A]
    k = 0
    while True:
        B, _, _ = O.gam_sweep(wl.idx, t, An, wl.dims, O.LOSS_POISSON_LOG, 0.1, 0.0, 1)
        D = B[0] - An[0]
        An[0] = B[0]
        k += 1
        if np.linalg.norm(D) <= 1e-3 * np.linalg.norm(B[0]):
            break
    assert k == c1[0]


# ------------------------------------------------------------------ CCD ----
def test_ccd_rank1_is_als():
    """Rank 1: coordinate minimization of the single column is the ALS
    update of each mode (Section 2.3), so one CCD++ sweep equals one ALS
    sweep from the same start (different arithmetic: residual contractions
    against the Omega-hat Gram and Cholesky solve)."""
    wl = W.random_tensor((9, 10, 8), 200, 55, rank=1)
    lam = 1e-3
    A = W.init_factors(wl.dims, 1, float(np.mean(wl.t)), 3, dtype=np.float64)
    Aa, _ = O.als_sweep(wl.idx, wl.t, A, wl.dims, lam)
    Ac, _ = O.ccd_sweep(wl.idx, wl.t, A, wl.dims, lam)
    for d in range(3):
        np.testing.assert_allclose(Ac[d], Aa[d], rtol=1e-10, atol=1e-13)


def test_ccd_monotone_stationary_and_residual():
    """Each coordinate update minimizes exactly, so the objective
    (sum (t - m)^2 + lam sum ||A||^2) never increases; right after a sweep
    the last updated column (r = R-1 of the last mode) has zero partial
    derivatives; the incrementally kept residual equals t - model."""
    wl = W.random_tensor((9, 10, 8), 200, 56, rank=3)
    lam = 1e-3
    A = W.init_factors(wl.dims, 4, float(np.mean(wl.t)), 5, dtype=np.float64)
    f_prev = O.objective(wl.idx, wl.t, A, O.LOSS_LS, lam)
    for _ in range(3):
        A, rho = O.ccd_sweep(wl.idx, wl.t, A, wl.dims, lam)
        f = O.objective(wl.idx, wl.t, A, O.LOSS_LS, lam)
        assert f <= f_prev * (1 + 1e-12)
        f_prev = f
        g = O.gradient(wl.idx, wl.t, A, O.LOSS_LS, lam, wl.dims)[2][:, 3]
        assert np.abs(g).max() < 1e-10 * max(1.0, np.abs(wl.t).max())
        np.testing.assert_allclose(rho, wl.t - O.tttp(wl.idx, None, A), rtol=0, atol=1e-12)


# ----------------------------------------------------------------- bf16 ----
def test_bf16_rne():
    exact = np.array([0.0, 1.0, -2.5, 0.15625, 2.0 ** 127 * 1.5, 2.0 ** -120])
    np.testing.assert_array_equal(O.bf16_round(exact), exact.astype(np.float32))
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert O.bf16_round(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: ties to even -> 1+2^-6
    assert O.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2000) * 10.0 ** rng.integers(-5, 5, 2000)
    r = O.bf16_round(x)
    # brute force: nearest bf16 among the neighbours of the truncated value
    f = x.astype(np.float32)
    u = f.view(np.uint32) & np.uint32(0xFFFF0000)
    cands = np.stack([u, u + np.uint32(0x10000)]).view(np.float32).astype(np.float64)
    d = np.abs(cands - f.astype(np.float64))
    best = np.where(d[0] < d[1], cands[0], cands[1])
    tie = d[0] == d[1]
    even = np.where((u >> 16) % 2 == 0, cands[0], cands[1])
    np.testing.assert_array_equal(r, np.where(tie, even, best))
