"""The epipolar loss as a torch.autograd.Function.

Forward and backward both come from the library's hand-written adjoint
(fm_epipolar_loss_grad): one call evaluates L = inv_Z * sum_n e_n^T W_n e_n
and dL/dparams together, as the paper's fused forward+backward kernel does
(Sec. 3.4); backward only scales the stored gradient by the incoming one.
No torch operator touches the loss arithmetic.
"""
from __future__ import annotations

import torch

from . import api


class EpipolarLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, scene: api.Scene, W36: torch.Tensor, inv_Z: float):
        loss, grad = api.epipolar_loss_grad(scene, W36, params.detach().contiguous(), inv_Z=inv_Z,
                                            want_grad=params.requires_grad)
        ctx.save_for_backward(grad if grad is not None else torch.empty(0, device=params.device))
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return (g.to(grad.dtype) * grad, None, None, None)


def epipolar_loss(params: torch.Tensor, scene: api.Scene, W36: torch.Tensor, inv_Z: float) -> torch.Tensor:
    """Differentiable epipolar loss (float64 scalar) of params [N,9] float32."""
    return EpipolarLoss.apply(params, scene, W36, inv_Z)
