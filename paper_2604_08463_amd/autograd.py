"""torch.autograd.Function around the hand-written adjoint of the spectral likelihood.

Forward calls ``cs_likelihood_grad`` once and keeps the per-cluster gradient; backward scales
it by the incoming gradient of each item (paper Sec. 3.3.1: the gradient comes from the GLS
residuals, not from differentiating through the solver).
"""

from __future__ import annotations

import torch

from ._lib import Problem


class CsLikelihood(torch.autograd.Function):
    """``F = CsLikelihood.apply(x, problem)``: x packed ``[Ktot]`` float64 -> ``F[B]``."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, problem: Problem):
        f, g, _, st = problem.cs_likelihood_grad(x.detach())
        ctx.save_for_backward(g, problem.param_item)
        ctx.mark_non_differentiable(st)
        return f, st

    @staticmethod
    def backward(ctx, g_f, g_st):
        g, item = ctx.saved_tensors
        return g_f.index_select(0, item) * g, None


def neg2logl(x: torch.Tensor, problem: Problem) -> torch.Tensor:
    """Differentiable ``-2 ln L_spec`` per item."""
    f, _ = CsLikelihood.apply(x, problem)
    return f
