"""torch.autograd.Function over the library's amplitude loss.

forward:  L = sum_j || |F(w o S_j u)| - sqrt(f_j) ||^2 (odp_amp_loss, no gradients)
backward: the spectra are recomputed by odp_amp_loss, which returns dL/du and
          dL/dw (dL/dRe + i dL/dIm, PyTorch's convention for real losses of
          complex tensors); nothing but the inputs is saved between the passes.
"""
from __future__ import annotations

import torch


class AmplitudeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, w: torch.Tensor, plan) -> torch.Tensor:
        u = u.contiguous()
        w = w.contiguous()
        loss, _, _ = plan.amp_loss(u, w, grad_u=False, grad_w=False)
        ctx.save_for_backward(u, w)
        ctx.plan = plan
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        u, w = ctx.saved_tensors
        need_u, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        _, gu, gw = ctx.plan.amp_loss(u, w, grad_u=need_u, grad_w=need_w)
        scale = grad_out.to(torch.float32)
        if gu is not None:
            gu = gu * scale
        if gw is not None:
            gw = gw * scale
        return gu, gw, None


def amplitude_loss(u: torch.Tensor, w: torch.Tensor, plan) -> torch.Tensor:
    """Differentiable amplitude loss of image u and probe w on a bound plan."""
    return AmplitudeLoss.apply(u, w, plan)
