"""The placement objective f = W~ + lambda * N (Eq. (7)) as a differentiable
torch function.

Forward evaluates the scalar loss only: density (Eq. (2)), the spectral
solve (Eqs. (9)-(11)) with the energy N = sum rho * psi (Eq. (6)) and the
weighted-average wirelength W~ (Eq. (3)), all in libfftpl kernels.  Nothing
the size of the grid is kept for the backward pass: only the positions are
saved, and backward recomputes the density and the spectral coefficients and
runs the gradient kernels (the exact derivative dN/dx of Section III-C and
dW~/dx), scaled by the incoming gradient.  This trades one more solve for
not holding psi (4 MiB at n = 1024) per pending backward.
"""
from __future__ import annotations

import torch

from . import fftpl


class _Objective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, plan, prob, lam, gamma):
        out4 = torch.empty(4, dtype=torch.float64, device=x.device)
        fftpl.eval(plan, prob, x, y, lam, gamma, "exact", None, None, out4)
        ctx.save_for_backward(x, y)
        ctx.plan, ctx.prob, ctx.lam, ctx.gamma = plan, prob, float(lam), float(gamma)
        ctx.mark_non_differentiable(out4)
        return out4[1] + ctx.lam * out4[0], out4

    @staticmethod
    def backward(ctx, g_loss, g_out4):
        x, y = ctx.saved_tensors
        gx = torch.empty_like(x)
        gy = torch.empty_like(y)
        out4 = torch.empty(4, dtype=torch.float64, device=x.device)
        fftpl.eval(ctx.plan, ctx.prob, x, y, ctx.lam, ctx.gamma, "exact", gx, gy, out4)
        s = g_loss.to(torch.float32)
        return gx * s, gy * s, None, None, None, None


def objective(x, y, plan: fftpl.Plan, prob: fftpl.Problem, lam: float, gamma: float):
    """Returns (loss, scalars): loss = W~ + lam * N as a float64 0-dim tensor
    differentiable in the float32 positions x, y [num_cells]; scalars =
    [N, W~, HPWL, tau] (not differentiable).  prob needs an atomic-free path
    (the default exchange index)."""
    if not prob.fast:
        raise ValueError("objective needs a Problem with an index (path 'xch' or 'slots')")
    return _Objective.apply(x, y, plan, prob, lam, gamma)
