"""Plain FP64 completion drivers built from the primitives in ``cp`` (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.
"""
import numpy as np

from . import cp


def als_sweep(idx, t, A, dims, lam):
    """One least-squares ALS sweep (Section 2.2; Section 4 ALS listing):
    modes in order 0..N-1 (block Gauss-Seidel, Appendix A); for mode n the
    right-hand sides are M = MTTKRP_n(t) and the new rows solve
    (G^(i) + lam I) x_i = M_i with G^(i) built from Omega-hat.  The current
    rows of mode n are not used (Newton step from a zero initial guess).
    Returns the new factor list and, per mode, (G, M, info) of that solve
    (G without lam, for the fast-loss identity).
    Pinned by: monotone objective decrease, vanishing gradient of the solved
    mode, the fast-loss identity, and ridge regression by lstsq."""
    A = [np.array(a, dtype=np.float64) for a in A]
    aux = []
    for n in range(len(A)):
        M = cp.mttkrp(idx, t, A, n, dims[n])
        G = cp.gram(idx, None, A, n, dims[n])
        X, info = cp.solve_rows(G, M, lam)
        A[n] = X
        aux.append((G, M, info))
    return A, aux


def als_fast_loss(t, A_n, G, M):
    """Least-squares loss after solving mode n, from that solve's left- and
    right-hand sides (Section 2.2 identity):
    sum t^2 + sum_i a_i^T G^(i) a_i - 2 sum_{i,r} a_ir M_ir."""
    A_n = np.asarray(A_n, dtype=np.float64)
    quad = float(np.einsum("ir,irs,is->", A_n, G, A_n))
    lin = float(np.sum(A_n * M))
    return float(np.sum(np.asarray(t, dtype=np.float64) ** 2)) + quad - 2.0 * lin


def _dot(X, Y):
    return float(sum(np.sum(np.asarray(x) * np.asarray(y)) for x, y in zip(X, Y)))


def pcg(apply_H, apply_Pinv, B, tol, kmax):
    """Preconditioned conjugate gradient on block vectors (lists of arrays),
    from x0 = 0.  Stops when the unpreconditioned residual norm, relative to
    the initial one, is at most ``tol`` or after ``kmax`` iterations
    (Section 5.6 / 5.7 stopping rule).  Inner products run over the
    concatenation of all blocks.  Returns (X, iterations, final rel. res.).
    Pinned by: convergence to numpy.linalg.solve on small SPD systems."""
    X = [np.zeros_like(b, dtype=np.float64) for b in B]
    Rr = [np.array(b, dtype=np.float64) for b in B]
    r0 = np.sqrt(_dot(Rr, Rr))
    if r0 == 0.0:
        return X, 0, 0.0
    Z = apply_Pinv(Rr)
    P = [z.copy() for z in Z]
    rz = _dot(Rr, Z)
    rel = 1.0
    k = 0
    while k < kmax:
        HP = apply_H(P)
        alpha = rz / _dot(P, HP)
        X = [x + alpha * p for x, p in zip(X, P)]
        Rr = [r - alpha * hp for r, hp in zip(Rr, HP)]
        k += 1
        rel = np.sqrt(_dot(Rr, Rr)) / r0
        if rel <= tol:
            break
        Z = apply_Pinv(Rr)
        rz_new = _dot(Rr, Z)
        beta = rz_new / rz
        rz = rz_new
        P = [z + beta * p for z, p in zip(Z, P)]
    return X, k, rel


def gn_step(idx, t, A, dims, loss, lam, tol, kmax):
    """One preconditioned Gauss-Newton iteration (Section 2.5 and its
    implementation in Section 4): solve H dx = -grad f by PCG with the
    implicit GN operator (weights phi'', diagonal shift 2 lam) and the
    block-diagonal preconditioner applied through Solve Factor (weights
    phi'', shift 2 lam); then take the full step A + dx (no line search)."""
    A = [np.array(a, dtype=np.float64) for a in A]
    m = cp.model_values(idx, A)
    w = cp.d2phi(t, m, loss)
    g = cp.gradient(idx, t, A, loss, lam, dims)
    B = [-x for x in g]
    lam2 = 2.0 * lam
    Gs = [cp.gram(idx, w, A, d, dims[d]) for d in range(len(A))]

    def apply_H(X):
        return cp.gn_matvec(idx, w, A, X, lam2, dims)

    def apply_Pinv(Rb):
        return [cp.solve_rows(Gs[d], Rb[d], lam2)[0] for d in range(len(A))]

    dX, iters, rel = pcg(apply_H, apply_Pinv, B, tol, kmax)
    return [a + dx for a, dx in zip(A, dX)], iters, rel


def gam_sweep(idx, t, A, dims, loss, lam, tol, max_inner):
    """One generalized alternating-minimization sweep (Section 2.2, general
    loss): modes in order 0..N-1; for mode n, Newton iterations on its rows
    with the other factors fixed.  Each iteration recomputes the model
    values m, phi'(t, m) and phi''(t, m), then for every row i solves
        (G_phi''^(i) + 2 lam I) d_i = -(MTTKRP_n(phi')_i + 2 lam u_i)
    (Hessian and gradient of Table 1 restricted to row i; the objective's
    regularizer lam ||A||^2 gives the 2 lam terms) and sets u_i <- u_i + d_i.
    A mode stops after ``max_inner`` iterations or once
    ||D||_F <= tol ||A_n||_F with D the whole step of that iteration and A_n
    the updated factor (Section 5.7's relative step tolerance, read over the
    factor matrix).  tol <= 0 always runs ``max_inner`` iterations.
    Returns the new factors, the inner iteration count per mode and the
    solve info of each mode's last iteration.
    Pinned by: least squares, where one Newton step from any start is the
    ALS solve; Poisson rows after converged inner iterations against a
    general-purpose minimizer of the row's objective written from phi."""
    A = [np.array(a, dtype=np.float64) for a in A]
    counts, infos = [], []
    for n in range(len(A)):
        k, info = 0, np.zeros(dims[n], dtype=np.int64)
        while k < max_inner:
            m = cp.model_values(idx, A)
            g = cp.mttkrp(idx, cp.dphi(t, m, loss), A, n, dims[n]) + 2.0 * lam * A[n]
            G = cp.gram(idx, cp.d2phi(t, m, loss), A, n, dims[n])
            D, info = cp.solve_rows(G, -g, 2.0 * lam)
            A[n] = A[n] + D
            k += 1
            if tol > 0 and np.linalg.norm(D) <= tol * np.linalg.norm(A[n]):
                break
        counts.append(k)
        infos.append(info)
    return A, counts, infos


def ccd_sweep(idx, t, A, dims, lam):
    """One least-squares coordinate-minimization sweep in the CCD++ order
    (Section 2.3): for each column r, for each mode n in turn, every entry
    u_ir of that column is set to its exact minimizer with all else fixed,
        u_ir = sum_e rho_e h_er / (lam + sum_e h_er^2)    (e in row i),
    with h_er the product of the other modes' column-r entries and
    rho = t - model + (column r's own rank-1 term), the residual without
    column r (it does not change while column r is updated).  After the
    column, rho drops the new rank-1 term.  Returns the new factors and the
    final residual t - model kept incrementally.
    Pinned by: R = 1 equals the ALS sweep; the objective never increases;
    the last updated column has zero partial derivatives; the incremental
    residual equals the recomputed one."""
    A = [np.array(a, dtype=np.float64) for a in A]
    N, R = len(A), A[0].shape[1]
    t = np.asarray(t, dtype=np.float64)
    rho = t - cp.model_values(idx, A)
    for r in range(R):
        cols = [a[:, r:r + 1] for a in A]
        rho = rho + cp.tttp(idx, None, cols)
        for n in range(N):
            cols = [a[:, r:r + 1] for a in A]
            num = cp.mttkrp(idx, rho, cols, n, dims[n])[:, 0]
            sq = [c * c for c in cols]
            den = lam + cp.mttkrp(idx, None, sq, n, dims[n])[:, 0]
            A[n][:, r] = num / den
        cols = [a[:, r:r + 1] for a in A]
        rho = rho - cp.tttp(idx, None, cols)
    return A, rho
