"""torch.autograd integration: F(Q) as a differentiable function of the vertices, Q and densities."""
from __future__ import annotations

import torch

from . import api


class PftFunction(torch.autograd.Function):
    """F = pft_forward_3d(verts); dL/dverts = pft_backward_3d(grad_F), dL/dQ from
    pft_backward_3d_regions with one region of density 1 when Q requires grad.

    For a complex output PyTorch hands backward dL/dReF + i dL/dImF, which is
    exactly the ``grad_out`` convention of the library's adjoint. Triangle
    indices are constants.
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
        need_v, _, need_q = ctx.needs_input_grad[:3]
        gv = gq = None
        if need_q:
            one = torch.ones(1, dtype=torch.float64, device=verts.device)
            gv, _, gq = api.backward_3d_regions(verts, tris, [0, tris.shape[0]], one, q, grad_F, mode=ctx.mode,
                                                need_verts=need_v, need_rho=False, need_q=True)
        elif need_v:
            gv = api.backward_3d(verts, tris, q, grad_F, mode=ctx.mode)
        return gv, None, gq, None


class PftRegionsFunction(torch.autograd.Function):
    """F = sum_j rho_j F_j (pft_forward_3d_regions); gradients to the vertices, the densities and Q
    from pft_backward_3d_regions, each only when required."""

    @staticmethod
    def forward(ctx, verts, rho, q, tris, region_offsets, mode="fp32c"):
        F = api.forward_3d_regions(verts, tris, region_offsets, rho, q, mode=mode)
        ctx.save_for_backward(verts, rho, q, tris)
        ctx.region_offsets = region_offsets
        ctx.mode = mode
        return F

    @staticmethod
    def backward(ctx, grad_F):
        verts, rho, q, tris = ctx.saved_tensors
        nv, nr, nq = ctx.needs_input_grad[:3]
        gv, gr, gq = api.backward_3d_regions(verts, tris, ctx.region_offsets, rho, q, grad_F, mode=ctx.mode,
                                             need_verts=nv, need_rho=nr, need_q=nq)
        return gv, gr, gq, None, None, None


def ft3d(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, mode: str = "fp32c") -> torch.Tensor:
    """Differentiable F(Q) of a closed triangle mesh."""
    return PftFunction.apply(verts, tris, q, mode)


class IntensityLossFunction(torch.autograd.Function):
    """L = sum_Q w (|F|^2 - I)^2 as a function of the vertices, with dL/dverts computed by the fused
    library call in the forward pass and scaled by the incoming gradient in the backward pass."""

    @staticmethod
    def forward(ctx, verts, tris, q, target, weight, mode="fp32c"):
        loss, gv = api.intensity_loss_3d(verts, tris, q, target, weight, mode=mode,
                                         need_grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(gv if gv is not None else torch.empty(0, device=verts.device))
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        (gv,) = ctx.saved_tensors
        if gv.numel() == 0:
            return None, None, None, None, None, None
        return grad_loss.to(gv.dtype) * gv, None, None, None, None, None


def fused_intensity_loss(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, target: torch.Tensor,
                         weight=None, mode: str = "fp32c") -> torch.Tensor:
    """Differentiable sum_Q w (|F|^2 - I)^2 of a closed mesh (one fused library call per evaluation)."""
    return IntensityLossFunction.apply(verts, tris, q, target, weight, mode)


def ft3d_regions(verts: torch.Tensor, tris: torch.Tensor, region_offsets, rho: torch.Tensor, q: torch.Tensor,
                 mode: str = "fp32c") -> torch.Tensor:
    """Differentiable F(Q) of a piecewise-constant density over closed regions."""
    return PftRegionsFunction.apply(verts, rho, q, tris, region_offsets, mode)


def intensity_loss(F: torch.Tensor, target: torch.Tensor, weight) -> torch.Tensor:
    """sum_Q w(Q) (|F(Q)|^2 - I(Q))^2 (plain torch elementwise ops on the GPU)."""
    inten = F.real * F.real + F.imag * F.imag
    return torch.sum(weight * (inten - target) ** 2)
