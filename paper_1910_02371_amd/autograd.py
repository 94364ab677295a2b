"""Differentiable completion objective with a hand-written adjoint.

``CPLoss.apply(ix, loss, lam, A_0, ..., A_{N-1})`` returns the float64 scalar
f = sum_Omega phi(t, m) + lam * sum_n ||A_n||_F^2 (eq. obj), evaluated by the
TTTP loss epilogue.  Its backward is the adjoint of Table 1 / Appendix A:
grad_d = MTTKRP_d(phi'(t, m)) + 2 lam A_d, computed by ``tt_gradient`` (the
model values are recomputed inside each mode's pass), then scaled by the
incoming gradient and returned in the factors' dtype.
"""
import torch

from . import tt


class CPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ix, loss, lam, *A):
        ctx.ix = ix
        ctx.loss = loss
        ctx.lam = float(lam)
        ctx.save_for_backward(*A)
        return tt.objective(ix, list(A), loss, lam)

    @staticmethod
    def backward(ctx, gout):
        A = ctx.saved_tensors
        G = tt.gradient(ctx.ix, list(A), ctx.loss, ctx.lam)
        grads = []
        for g, a in zip(G, A):
            if gout is not None:
                g = g * gout.to(g.dtype)
            grads.append(g.to(a.dtype))
        return (None, None, None) + tuple(grads)


def cp_loss(ix, A, loss="ls", lam=0.0):
    return CPLoss.apply(ix, loss, lam, *A)
