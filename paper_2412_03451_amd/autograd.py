"""torch.autograd front end of the splat: depth and normal maps as a
differentiable function of the plane parameters (Sec. 3.2, Eq. 4-13).

The forward keeps no per-pixel state.  What the backward needs beyond the
inputs is the projection records and the depth-sorted tile lists, which live
in the renderer's workspace (O(pairs), not O(pixels x M)); the backward
kernel recomputes each pixel's compositing sequence from them.  If the
workspace was reused for another render in between, the backward projects
and bins again from the saved inputs first (same bits: both are
deterministic functions of the inputs).
"""

from __future__ import annotations

import torch

from .splat import Renderer


class PlaneSplatFn(torch.autograd.Function):
    """(center [K,3], quat [K,4], radii [K,4], lam [1]) -> (depth [P], normal [3P])
    for the jobs of `renderer`."""

    @staticmethod
    def forward(ctx, center, quat, radii, lam, renderer: Renderer):
        center, quat, radii = center.contiguous(), quat.contiguous(), radii.contiguous()
        renderer.project(center, quat, radii, lam)
        renderer.bin()
        D, N = renderer.forward()
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.save_for_backward(center, quat, radii, lam)
        return D, N

    @staticmethod
    def backward(ctx, gD, gN):
        center, quat, radii, lam = ctx.saved_tensors
        r: Renderer = ctx.renderer
        if r.generation != ctx.generation:
            r.project(center, quat, radii, lam)
            r.bin()
        if gD is None:
            gD = torch.zeros(r.n_pixels, dtype=torch.float32, device=center.device)
        if gN is None:
            gN = torch.zeros(3 * r.n_pixels, dtype=torch.float32, device=center.device)
        gc, gq, gr = r.backward(center, quat, radii, lam, gD.contiguous(), gN.contiguous())
        return gc, gq, gr, None, None


class PlaneSplatListsFn(torch.autograd.Function):
    """The list-storing variant: the forward keeps each pixel's committed
    hits (list position, a*, transmittance; M entries per pixel) for the
    backward.  Same values and gradients as PlaneSplatFn; kept for the memory
    comparison."""

    @staticmethod
    def forward(ctx, center, quat, radii, lam, renderer: Renderer):
        center, quat, radii = center.contiguous(), quat.contiguous(), radii.contiguous()
        renderer.project(center, quat, radii, lam)
        renderer.bin()
        D, N, lists = renderer.forward_lists()
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.save_for_backward(center, quat, radii, lam, *lists)
        return D, N

    @staticmethod
    def backward(ctx, gD, gN):
        center, quat, radii, lam, pos, a, T, cnt = ctx.saved_tensors
        r: Renderer = ctx.renderer
        if r.generation != ctx.generation:
            r.project(center, quat, radii, lam)
            r.bin()
        if gD is None:
            gD = torch.zeros(r.n_pixels, dtype=torch.float32, device=center.device)
        if gN is None:
            gN = torch.zeros(3 * r.n_pixels, dtype=torch.float32, device=center.device)
        gc, gq, gr = r.backward_lists(center, quat, radii, lam, gD.contiguous(), gN.contiguous(), (pos, a, T, cnt))
        return gc, gq, gr, None, None


def plane_splat(center, quat, radii, lam, renderer: Renderer):
    """Differentiable render of the renderer's jobs; see PlaneSplatFn."""
    if not torch.is_tensor(lam):
        lam = torch.tensor([float(lam)], dtype=torch.float32, device=center.device)
    return PlaneSplatFn.apply(center, quat, radii, lam, renderer)
