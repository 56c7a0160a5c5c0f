"""torch.autograd integration: F(Q) as a differentiable function of the vertices."""
from __future__ import annotations

import torch

from . import api


class PftFunction(torch.autograd.Function):
    """F = pft_forward_3d(verts); dL/dverts = pft_backward_3d(grad_F).

    For a complex output PyTorch hands backward dL/dReF + i dL/dImF, which is
    exactly the ``grad_out`` convention of the library's adjoint. Gradients
    flow to the vertices only (triangle indices and Q are constants).
    """

    @staticmethod
    def forward(ctx, verts, tris, q, mode="fp32c"):
        F = api.forward_3d(verts, tris, q, mode=mode)
        ctx.save_for_backward(verts, tris, q)
        ctx.mode = mode
        return F

    @staticmethod
    def backward(ctx, grad_F):
        verts, tris, q = ctx.saved_tensors
        g = api.backward_3d(verts, tris, q, grad_F, mode=ctx.mode)
        return g, None, None, None


def ft3d(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, mode: str = "fp32c") -> torch.Tensor:
    """Differentiable F(Q) of a closed triangle mesh."""
    return PftFunction.apply(verts, tris, q, mode)


def intensity_loss(F: torch.Tensor, target: torch.Tensor, weight) -> torch.Tensor:
    """sum_Q w(Q) (|F(Q)|^2 - I(Q))^2 (plain torch elementwise ops on the GPU)."""
    inten = F.real * F.real + F.imag * F.imag
    return torch.sum(weight * (inten - target) ** 2)
