"""Differentiable windowed SSD of the deformation, and gradient refinement.

``PivWarpSSD`` wraps the library's forward (per-window sum of squared
differences between A and B deformed by the interpolated node field U) and
its hand-written adjoint with respect to U as a torch.autograd.Function.
``refine`` runs preconditioned gradient steps U <- U - dL/dU / (D + lambda)
with D the Gauss-Newton diagonal returned by the adjoint.

This is an addition of this library (the paper refines with a Gaussian fit
on the correlation stencil only); both run on the same plan geometry so the
two estimates can be compared node by node.
"""
from __future__ import annotations

from typing import Tuple

import torch

from .api import Plan


class PivWarpSSD(torch.autograd.Function):
    """loss[n][ny][nx] = sum over each window of (B(p + u(p)) - A(p))^2.

    Differentiable in U only (A and B are data).  The plan must be a
    ``dtype="f32"`` plan with the images' size and the grid of U.
    """

    @staticmethod
    def forward(ctx, A: torch.Tensor, B: torch.Tensor, U: torch.Tensor, plan: Plan) -> torch.Tensor:
        A, B, U = A.contiguous(), B.contiguous(), U.contiguous()
        loss = plan.ssd_forward(A, B, U)
        ctx.save_for_backward(A, B, U)
        ctx.plan = plan
        return loss

    @staticmethod
    def backward(ctx, g_loss: torch.Tensor):
        A, B, U = ctx.saved_tensors
        gU, _ = ctx.plan.ssd_backward(A, B, U, g_loss.contiguous(), want_diag=False)
        return None, None, gU, None


def warp_ssd(A, B, U, plan: Plan) -> torch.Tensor:
    return PivWarpSSD.apply(A, B, U, plan)


def refine(plan: Plan, A: torch.Tensor, B: torch.Tensor, U0: torch.Tensor, steps: int = 10,
           lam_rel: float = 1e-3, tau: float = 4.0 / 9.0) -> Tuple[torch.Tensor, torch.Tensor]:
    """`steps` diagonally preconditioned gradient steps on the total windowed
    SSD, from U0 [n][2][ny][nx] (left unchanged):
    U <- U - tau dL/dU / (D + lambda), with D the Gauss-Newton diagonal and
    lambda = lam_rel * mean(D) per pair, all on the device (piv_ssd_refine).

    The diagonal ignores that neighbouring nodes share pixels: when they
    err together, the step overshoots by sum(w)/sum(w^2) over a node's
    support, which is (3/2)^2 = 9/4 for bilinear hat weights; tau = 4/9
    removes that factor.  Returns the refined field and the device tensor
    [n][steps + 1] of total losses before each step and after the last."""
    U = U0.detach().clone().contiguous()
    hist = torch.empty((U.shape[0], steps + 1), dtype=torch.float32, device=U.device)
    plan.ssd_refine(A, B, U, steps=steps, tau=tau, lam_rel=lam_rel, hist=hist)
    return U, hist
