"""Plain FP64 definitions of the sparse CP-completion primitives (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Notation follows the paper: a sparse tensor with observed index set Omega of
m nonzeros, stored as N index arrays ``idx[n]`` (0-based, length m) and values
``s`` (or ``t`` for observed data); factor matrices ``A[n]`` of shape
(I_n, R); the CP model m_e = sum_r prod_n A[n][i_n(e), r] (eq. 1/2, and the
order-N form of Appendix A).
"""
import numpy as np
import scipy.linalg

LOSS_LS = 0
LOSS_POISSON_LOG = 1


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# Index: stable counting sort of the nonzeros by one mode (Section 3.4).
# --------------------------------------------------------------------------
def mode_index(idx, n, I_n):
    """Counting-sort index of one mode (see ``build_index``)."""
    N = len(idx)
    key = np.asarray(idx[n], dtype=np.int64)
    cnt = np.bincount(key, minlength=int(I_n)).astype(np.int64)
    ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    perm = np.argsort(key, kind="stable").astype(np.int64)
    rows = np.flatnonzero(cnt).astype(np.int64)
    other = {p: np.asarray(idx[p], dtype=np.int64)[perm]
             for p in range(N) if p != n}
    return dict(cnt=cnt, ptr=ptr, perm=perm, rows=rows, key=key[perm],
                other=other)


def build_index(idx, dims):
    """Per mode n: counts, row pointers, stable sort permutation, nonzero rows
    and the other modes' indices in sorted order.

    Section 3.4 sorts the local nonzeros by the mode-n index with a counting
    sort, which is stable: equal keys keep their original (COO) order.  That
    is exactly ``argsort(kind='stable')``.

    Returns a list over modes of dicts with keys ``cnt`` (I_n,), ``ptr``
    (I_n+1,) int64, ``perm`` (m,) int64 (sorted position -> COO position),
    ``rows`` (nonzero rows), ``key`` (sorted mode-n indices) and ``other``
    (dict p -> idx[p][perm]).
    Pinned by: bincount/cumsum/argsort library routines plus brute-force
    checks of sortedness and stability in tests.
    """
    return [mode_index(idx, n, dims[n]) for n in range(len(idx))]


# --------------------------------------------------------------------------
# TTTP (Section 3.3): x_e = s_e * sum_r prod_{n in P} A[n][i_n(e), r].
# --------------------------------------------------------------------------
def tttp(idx, s, A):
    """Tensor-times-tensor product.

    ``A`` is a list of length N whose entries are (I_n, R) matrices, (I_n,)
    vectors (treated as R = 1) or ``None``; a ``None`` mode is skipped, so the
    product runs only over the provided modes (Section 3.3).  ``s`` may be
    ``None`` for the unit-valued pattern tensor Omega-hat.
    Pinned by: dense masked CP reconstruction (brute force), the SDDMM case
    S * (U V^T) for N = 2, and all-ones factors giving x = s * R.
    """
    mats = [(n, _f64(a).reshape(len(a), -1)) for n, a in enumerate(A)
            if a is not None]
    if not mats:
        raise ValueError("TTTP needs at least one factor")
    m = len(idx[0])
    R = mats[0][1].shape[1]
    prod = np.ones((m, R))
    for n, a in mats:
        prod = prod * a[np.asarray(idx[n], dtype=np.int64), :]
    x = prod.sum(axis=1)
    if s is not None:
        x = _f64(s) * x
    return x


# --------------------------------------------------------------------------
# Elementwise loss and its derivatives in the model value m (eq. deriv_tnsr).
# --------------------------------------------------------------------------
def phi(t, m, loss):
    """phi(t, m): least squares (t - m)^2 (Section 2.1) or the Poisson
    log-link loss exp(m) - t m (Section 5.7; the log t! constant is dropped).
    Pinned by: closed-form values and finite differences of dphi/d2phi."""
    t, m = _f64(t), _f64(m)
    if loss == LOSS_LS:
        return (t - m) ** 2
    if loss == LOSS_POISSON_LOG:
        return np.exp(m) - t * m
    raise ValueError(loss)


def dphi(t, m, loss):
    """d phi / d m: 2 (m - t) for least squares, exp(m) - t for Poisson
    log link (eq. deriv_tnsr applied to the two losses)."""
    t, m = _f64(t), _f64(m)
    if loss == LOSS_LS:
        return 2.0 * (m - t)
    if loss == LOSS_POISSON_LOG:
        return np.exp(m) - t
    raise ValueError(loss)


def d2phi(t, m, loss):
    """d^2 phi / d m^2: the constant 2 for least squares, exp(m) for Poisson
    log link."""
    t, m = _f64(t), _f64(m)
    if loss == LOSS_LS:
        return np.full(np.broadcast(t, m).shape, 2.0)
    if loss == LOSS_POISSON_LOG:
        return np.exp(m)
    raise ValueError(loss)


# --------------------------------------------------------------------------
# MTTKRP (Section 2.2 right-hand sides; Section 3.2; Appendix A gradient).
# --------------------------------------------------------------------------
def _hadamard_rows(idx, A, n):
    """h_e = Hadamard product over modes p != n of A[p][i_p(e), :] (m, R)."""
    N = len(idx)
    m = len(idx[0])
    R = None
    h = None
    for p in range(N):
        if p == n:
            continue
        a = _f64(A[p]).reshape(len(A[p]), -1)
        R = a.shape[1]
        g = a[np.asarray(idx[p], dtype=np.int64), :]
        h = g if h is None else h * g
    if h is None:
        h = np.ones((m, R if R else 1))
    return h


def mttkrp(idx, s, A, n, I_n):
    """Y[i, r] = sum over nonzeros e with i_n(e) = i of
    s_e * prod_{p != n} A[p][i_p(e), r].

    ``s`` = None means Omega-hat (unit values).  ``A[n]`` is ignored.
    Pinned by: the explicit Khatri-Rao product of the dense unfolding (brute
    force), and sum_e TTTP_e = <A_n, MTTKRP_n> for every n.
    """
    h = _hadamard_rows(idx, A, n)
    if s is not None:
        h = h * _f64(s)[:, None]
    Y = np.zeros((int(I_n), h.shape[1]))
    np.add.at(Y, np.asarray(idx[n], dtype=np.int64), h)
    return Y


# --------------------------------------------------------------------------
# Solve Factor (Section 3.4): per-row Gram build and SPD solve.
# --------------------------------------------------------------------------
def row_design(idx, A, n, ix_n, i):
    """H_i: the rows h_e of the nonzeros in row i of mode n, in sorted order,
    and their COO positions.  ``ix_n`` is ``build_index(...)[n]``."""
    sel = ix_n["perm"][ix_n["ptr"][i]:ix_n["ptr"][i + 1]]
    sub = [np.asarray(idx[p])[sel] for p in range(len(idx))]
    return _hadamard_rows(sub, A, n), sel


def gram(idx, w, A, n, I_n, rows=None):
    """G^(i) = sum_{e in row i} w_e h_e h_e^T for each row i (Section 3.4's
    left-hand sides; Section 2.2 with w = Omega-hat).  Computed directly as
    H_i^T diag(w) H_i, with no square root of w, so any sign of w is allowed.

    Returns an (len(rows), R, R) array.  Pinned by: explicit H_i products,
    the quadratic-form identity sum_i a_i^T G^(i) a_i = sum_e w_e m_e^2, and
    the Omega = all-entries case where every G^(i) equals the Hadamard
    product of the other factors' Gram matrices.
    """
    ix_n = mode_index(idx, n, I_n)
    if rows is None:
        rows = np.arange(int(I_n))
    R = next(_f64(A[p]).reshape(len(A[p]), -1).shape[1]
             for p in range(len(idx)) if p != n)
    out = np.zeros((len(rows), R, R))
    for t, i in enumerate(rows):
        H, sel = row_design(idx, A, n, ix_n, int(i))
        ww = np.ones(len(sel)) if w is None else _f64(w)[sel]
        out[t] = H.T @ (ww[:, None] * H)
    return out


def cholesky_info(S):
    """LAPACK potrf convention: 0 if S is positive definite, else the order k
    of the first leading minor that is not positive.  Plain
    Cholesky-Banachiewicz loop (row by row)."""
    S = _f64(S)
    R = S.shape[0]
    L = np.zeros_like(S)
    for i in range(R):
        for j in range(i + 1):
            acc = S[i, j] - np.dot(L[i, :j], L[j, :j])
            if i == j:
                if not acc > 0.0:
                    return i + 1
                L[i, i] = np.sqrt(acc)
            else:
                L[i, j] = acc / L[j, j]
    return 0


def solve_rows(G, M, lam):
    """x_i = (G^(i) + lam I)^{-1} M_i per row by Cholesky and two triangular
    solves (the POSV of Section 3.4).  A row whose matrix is not positive
    definite gets x_i = 0 and info_i = the failing leading-minor order.
    Pinned by: normwise backward error, ridge regression by lstsq, and the
    R = 1 coordinate-descent closed form of Section 2.3."""
    G = _f64(G)
    M = _f64(M)
    nrow, R, _ = G.shape
    X = np.zeros((nrow, R))
    info = np.zeros(nrow, dtype=np.int32)
    eye = np.eye(R)
    for i in range(nrow):
        S = G[i] + lam * eye
        try:
            L = np.linalg.cholesky(S)
        except np.linalg.LinAlgError:
            info[i] = cholesky_info(S)
            continue
        y = scipy.linalg.solve_triangular(L, M[i], lower=True)
        X[i] = scipy.linalg.solve_triangular(L.T, y, lower=False)
    return X, info


def solve_factor(idx, w, A, n, I_n, M, lam):
    """Solve Factor (Section 3.4): for every row i of mode n solve
    (G^(i) + lam I) x_i = M_i with G^(i) the weighted Gram of that row.
    ``lam`` is added exactly as given (least-squares ALS passes lambda, the
    Gauss-Newton preconditioner passes 2 lambda).  Rows without nonzeros
    have G = 0, so x = M / lam (info = 1 when lam = 0)."""
    G = gram(idx, w, A, n, I_n)
    return solve_rows(G, M, lam)


# --------------------------------------------------------------------------
# Objective, gradient and Gauss-Newton operator (Section 2.5, Appendix A).
# --------------------------------------------------------------------------
def model_values(idx, A):
    return tttp(idx, None, A)


def objective(idx, t, A, loss, lam):
    """f = sum_Omega phi(t, m) + lam * sum_n ||A_n||_F^2 (eq. obj)."""
    m = model_values(idx, A)
    return float(np.sum(phi(t, m, loss)) +
                 lam * sum(float(np.sum(_f64(a) ** 2)) for a in A))


def rmse(idx, t, A):
    """sqrt(mean over Omega of (t - m)^2) on the training entries."""
    m = model_values(idx, A)
    return float(np.sqrt(np.mean((_f64(t) - m) ** 2)))


def gradient(idx, t, A, loss, lam, dims):
    """grad_{A_d} f = MTTKRP_d(phi'(t, m)) + 2 lam A_d (Table 1 gradient row;
    Appendix A).  Pinned by central finite differences of ``objective``."""
    m = model_values(idx, A)
    d1 = dphi(t, m, loss)
    return [mttkrp(idx, d1, A, d, dims[d]) + 2.0 * lam * _f64(A[d])
            for d in range(len(A))]


def jvp(idx, A, X):
    """z = J x: the directional derivative of the model values in the
    direction (X_1..X_N): sum_p TTTP with slot p replaced by X_p."""
    N = len(A)
    z = np.zeros(len(idx[0]))
    for p in range(N):
        Ap = list(A)
        Ap[p] = X[p]
        z += tttp(idx, None, Ap)
    return z


def gn_matvec(idx, w, A, X, lam2, dims):
    """Gauss-Newton operator (Section 2.5 without the phi' terms; Appendix A
    first Hessian term): y_d = J_d^T diag(w) J x + lam2 X_d, with w = phi''
    per nonzero.  J_d^T applied to a per-nonzero vector is MTTKRP_d
    (Section 2.5: TTTP followed by MTTKRP).  Pinned by the explicit Jacobian
    on tiny tensors, symmetry and positive semidefiniteness."""
    z = jvp(idx, A, X)
    wz = _f64(w) * z
    return [mttkrp(idx, wz, A, d, dims[d]) + lam2 * _f64(X[d])
            for d in range(len(A))]


def newton_matvec(idx, t, A, X, lam2, dims, loss):
    """Full Hessian-vector product of the objective (Section 2.5 with the
    phi' terms of the off-diagonal blocks; Appendix A): the Gauss-Newton
    operator with w = phi'' plus, for every block d,
        sum_e phi'_e * sum_{p != d} X_p[i_p] * prod_{q != d, p} A_q[i_q],
    i.e. the MTTKRP of phi' with the factor of one other mode p replaced by
    the direction X_p, summed over p.  lam2 is the regularizer's Hessian
    (2 lambda).
    Pinned by: central differences of the oracle gradient in the direction
    X, symmetry, and equality with the GN operator where phi' = 0."""
    m = model_values(idx, A)
    y = gn_matvec(idx, d2phi(t, m, loss), A, X, lam2, dims)
    d1 = dphi(t, m, loss)
    for d in range(len(A)):
        for p in range(len(A)):
            if p == d:
                continue
            Ap = list(A)
            Ap[p] = X[p]
            y[d] = y[d] + mttkrp(idx, d1, Ap, d, dims[d])
    return y
