"""ln L(lambda) as a differentiable torch function for gradient-based samplers.

LnL.apply(lam, ctx, events, prec) takes lam as a float64 device tensor
[B, 14] (H0, Om, Xi0, n, alpha, beta, mmin, mmax, mu_g, sigma_g, lambda_g,
gamma, kappa, z_p) and returns ln L [B].  The forward pass calls
chimera_lnl_grad, which evaluates ln L and its adjoint in one launch sequence;
backward scales the stored gradient by the incoming one.  mmin and mmax are
edges of the mass support and get zero gradient (ln L jumps when a sample
crosses them); a point whose ln L is not finite gets NaN.
"""
from __future__ import annotations

import torch

from . import chimera

# columns of lambda that the adjoint differentiates, in its output order
GRAD_COLUMNS = (0, 1, 2, 3, 4, 5, 8, 9, 10, 11, 12, 13)


class LnL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, context: "chimera.Context", events: "chimera.EventSet",
                prec: int = chimera.CHIMERA_FP64):
        lam_c = lam.detach().contiguous()
        lnl, grad = context.lnl_grad(events, lam_c, prec)
        full = torch.zeros(lam_c.shape, dtype=torch.float64, device=lam_c.device)
        full[:, list(GRAD_COLUMNS)] = grad
        ctx.save_for_backward(full)
        return lnl

    @staticmethod
    def backward(ctx, g_out):
        (full,) = ctx.saved_tensors
        return g_out[:, None] * full, None, None, None


def lnl(lam, context, events, prec=chimera.CHIMERA_FP64):
    """ln L [B] of lam [B, 14] with autograd support."""
    return LnL.apply(lam, context, events, prec)
