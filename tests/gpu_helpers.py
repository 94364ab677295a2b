"""Shared helpers of the GPU parity tests: device transfer and the error
measures used against the FP64 oracle.

Tolerance convention (elementwise): |x_gpu - x_ref| <= tau * x_abs, where
x_abs is the same expression evaluated on absolute values, so cancellation
does not inflate the allowed error.  tau = 1e-12 for FP64 kernels, 1e-5 for
FP32 kernels (and for BF16-stored factors compared with the oracle on the
same rounded factors), 2e-2 for BF16 against the unrounded factors."""
import numpy as np
import torch

import oracle as O

TAU = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}
TAU_BF16_VS_F32 = 2e-2
TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def dev_idx(idx):
    return [torch.as_tensor(np.asarray(i, dtype=np.int32)).cuda() for i in idx]


def dev_vals(t, form):
    dt = torch.float64 if form == "f64" else torch.float32
    return torch.as_tensor(np.asarray(t)).to(dt).cuda()


def dev_factor(a, form):
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(TORCH_DT[form]).cuda()


def host(t):
    if isinstance(t, (list, tuple)):
        return [host(x) for x in t]
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype != torch.bfloat16 else \
        t.detach().float().to(torch.float64).cpu().numpy()


def stored_values(t, form):
    """Observed values as the GPU sees them (float32 for the f32/bf16 forms)."""
    t = np.asarray(t)
    return t.astype(np.float64) if form == "f64" else t.astype(np.float32).astype(np.float64)


def stored_factors(A, form):
    """Factors as stored on the GPU, back in float64 (bf16: RNE-rounded)."""
    if form == "f64":
        return [np.asarray(a, dtype=np.float64) for a in A]
    if form == "f32":
        return [np.asarray(a, dtype=np.float32).astype(np.float64) for a in A]
    return [O.bf16_round(a) for a in A]


def assert_close_abs(gpu, ref, ref_abs, tau, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(gpu - ref)
    bound = tau * np.asarray(ref_abs, dtype=np.float64) + 1e-300
    ratio = err / bound
    worst = float(np.max(ratio)) if ratio.size else 0.0
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite GPU values"
    assert worst <= 1.0, (f"{what}: error {float(np.max(err)):.3e} exceeds tau*|x|_abs "
                          f"(worst ratio {worst:.3f}, tau={tau})")
    return worst


def backward_error(G, lam, X, M):
    """Normwise backward error of each row solve, max over rows."""
    worst = 0.0
    R = G.shape[1]
    for i in range(G.shape[0]):
        S = G[i] + lam * np.eye(R)
        num = np.linalg.norm(S @ X[i] - M[i])
        den = np.linalg.norm(S, 2) * np.linalg.norm(X[i]) + np.linalg.norm(M[i])
        worst = max(worst, num / den if den > 0 else num)
    return worst


def loss_abs(t, m, m_abs, loss, what):
    """The absolute-value form of an elementwise loss map at the model value
    m, against which its rounding error is measured: each operation of the
    map evaluated on absolute values, with the model value's own error
    (bounded relative to m_abs, the model on absolute factors) carried
    through the map's slope.
      least squares: resid |t| + m_abs, phi (|t| + m_abs)^2,
                     phi' 2 (|t| + m_abs), phi'' 2;
      Poisson log link (e = exp(m)): resid |t| + m_abs,
                     phi e (1 + m_abs) + |t| m_abs, phi' e (1 + m_abs) + |t|,
                     phi'' e (1 + m_abs)."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    m = np.asarray(m, dtype=np.float64)
    m_abs = np.asarray(m_abs, dtype=np.float64)
    if what == "resid":
        return t + m_abs
    if loss == O.LOSS_LS:
        return {"phi": (t + m_abs) ** 2, "dphi": 2.0 * (t + m_abs),
                "d2phi": np.full(np.broadcast(t, m).shape, 2.0)}[what]
    e = np.exp(m) * (1.0 + m_abs)
    return {"phi": e + t * m_abs, "dphi": e + t, "d2phi": e}[what]


def rounded_abs(ref, ref_abs, tau, rel_round):
    """Absolute expression for a result within tau * ref_abs that is then
    rounded with relative error rel_round (e.g. 2^-8 for bf16 RNE): the
    bound tau * ref_abs + rel_round * (|ref| + tau * ref_abs), written as
    tau * (returned value)."""
    ref = np.abs(np.asarray(ref, dtype=np.float64))
    ref_abs = np.asarray(ref_abs, dtype=np.float64)
    return ref_abs * (1.0 + rel_round) + ref * (rel_round / tau)
