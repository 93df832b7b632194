"""torch.autograd.Function over the library's reverse-mode adjoint.

LogContribution.apply(scene, L, u) returns log(p(u) + eps) for a batch of
primary-sample points u (n x d CUDA float32); its backward multiplies the
incoming gradient by the score grad_u log(p + eps) that dr_eval_logp_grad
computed in the same kernel as the forward value.
"""
from __future__ import annotations

import torch

from . import dr


class LogContribution(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene: "dr.Scene", L: int, u: torch.Tensor, eps: float = 1e-8):
        _, logp, g, _ = scene.eval_logp_grad(L, u.detach(), eps=eps, grad=True)
        ctx.save_for_backward(g)
        return logp

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return None, None, grad_out[:, None] * g, None
