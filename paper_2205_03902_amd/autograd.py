"""torch.autograd wrapper around the fused loss-and-gradient pass (ms_adjoint).

The forward pass runs the multislice model, the amplitude residual and the
hand-written adjoint in one call and caches the gradients.  ms_adjoint returns
the paper's generalised Wirtinger gradient dL/d conj(z) (Sec. 3.2); PyTorch's
complex autograd expects twice that for a real loss, so backward scales by 2.
"""
from __future__ import annotations

import torch

from .abi import Plan


class MultisliceAmplitudeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, probe: torch.Tensor, slices: torch.Tensor, plan: Plan, measured: torch.Tensor):
        loss, gs, gp = plan.adjoint(probe.detach().contiguous(), slices.detach().contiguous(), measured,
                                    want_probe=ctx.needs_input_grad[0])
        ctx.save_for_backward(gs, gp if gp is not None else torch.empty(0, device=slices.device))
        ctx.has_probe = gp is not None
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        gs, gp = ctx.saved_tensors
        scale = 2.0 * grad_out.to(torch.float32)
        g_probe = (gp * scale) if ctx.has_probe else None
        g_slices = gs * scale if ctx.needs_input_grad[1] else None
        return g_probe, g_slices, None, None


def amplitude_loss(plan: Plan, probe: torch.Tensor, slices: torch.Tensor, measured: torch.Tensor) -> torch.Tensor:
    """L = sum_s sum_k (sqrt(I_k^s) - |F E_M^s|_k)^2 as a differentiable float64 scalar."""
    return MultisliceAmplitudeLoss.apply(probe, slices, plan, measured)
