"""torch.autograd.Function around the fused HIP kernels.

forward:  J2[c] for every curve (FP64), from the J-only kernel.
backward: the adjoint kernel recomputes the residual, the physical fields and
          every transform from the saved state (nothing but the state is kept
          between the passes) and writes upstream[c] * dJ2/dstate in one pass.

The gradient is taken with respect to the free coordinates: the pinned
endpoint rows and the imaginary part of mode 0 receive zero.
"""
from __future__ import annotations

import torch

from .problem import Problem


class KSCurveJ2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state: torch.Tensor, prob: Problem):
        ctx.prob = prob
        ctx.save_for_backward(state)
        return prob.eval_J(state if state.is_contiguous() else state.contiguous())

    @staticmethod
    def backward(ctx, gJ2: torch.Tensor):
        (state,) = ctx.saved_tensors
        prob: Problem = ctx.prob
        scale = gJ2 if gJ2.dtype == torch.float64 else gJ2.to(torch.float64)
        if not scale.is_contiguous():  # e.g. the expanded upstream of a sum
            scale = scale.contiguous()
        grad, _ = prob.eval_grad(state if state.is_contiguous() else state.contiguous(),
                                 scale=scale, want_J2=False)
        return grad, None


def curve_J2(state: torch.Tensor, prob: Problem) -> torch.Tensor:
    """Differentiable J2 per curve."""
    return KSCurveJ2.apply(state, prob)
