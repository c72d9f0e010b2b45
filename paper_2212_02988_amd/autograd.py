"""PyTorch autograd wrapper of the renderer and its hand-written adjoint.

The emission of App. B is differentiable almost everywhere: with the hit
sample k* of each ray held fixed, depth and colour are smooth functions of
the voxel means and of the pose.  ``RenderFn`` runs ``prism_render`` in the
forward pass (keeping k* per ray, nothing else) and ``prism_render_vjp`` in
the backward pass, which recomputes the two bracketing samples of each ray
and scatters the gradient into the voxel means with atomic adds.

Gradients w.r.t. the pose are taken in the tangent delta = (dt, dtheta) of a
left perturbation, t <- t + dt, R <- Exp(dtheta) R (prism_pose_retract folds
delta into the base poses), and are exact at delta = 0.
"""
from __future__ import annotations

from typing import Tuple

import torch

from . import prism as P


class RenderFn(torch.autograd.Function):
    """(mean_planes [4, n^3] FP32 brick order, delta [F, 6]) -> (depth [F,H,W], rgb [F,H,W,3]).

    ``mean_planes`` must be the mean planes of ``vmap`` (``vmap.mean_planes()``,
    an FP32 map): the renderer reads the map buffer itself.  The forward pass
    refreshes the map's brick summary first, so in-place updates of the
    planes between calls are always seen."""

    @staticmethod
    def forward(ctx, mean_planes: torch.Tensor, delta: torch.Tensor, vmap: P.VoxelMap, grid: P.Grid,
                cam: P.Camera, poses: torch.Tensor):
        if mean_planes.data_ptr() != vmap.mean_planes().data_ptr():
            raise P.PrismError("mean_planes must be vmap.mean_planes()")
        vmap.refresh()
        # the perturbation delta folded into the base poses by the library's
        # retraction (t + dt, Exp(dtheta) R)
        p = P.pose_retract(poses.contiguous(), delta.detach().to(torch.float64).contiguous())
        out = P.render(grid, vmap, cam, p, hit_k=True)
        ctx.save_for_backward(out["hit_k"], p)
        ctx.vmap, ctx.grid, ctx.cam = vmap, grid, cam
        ctx.delta_dtype = delta.dtype
        ctx.mark_non_differentiable(out["mask"])
        return out["depth"], out["rgb"], out["mask"]

    @staticmethod
    def backward(ctx, g_depth, g_rgb, g_mask):
        hit_k, p = ctx.saved_tensors
        g_depth = torch.zeros_like(hit_k, dtype=torch.float32) if g_depth is None else g_depth.contiguous().float()
        if g_rgb is None:
            g_rgb = torch.zeros(hit_k.shape + (3,), dtype=torch.float32, device=hit_k.device)
        g_rgb = g_rgb.contiguous().float()
        gm, gp = P.render_vjp(ctx.grid, ctx.vmap, ctx.cam, p, hit_k, g_depth, g_rgb)
        return gm, gp.to(ctx.delta_dtype), None, None, None, None


def render(vmap: P.VoxelMap, cam: P.Camera, poses: torch.Tensor, delta: torch.Tensor,
           mean_planes: torch.Tensor | None = None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Differentiable render of ``vmap`` at ``poses`` perturbed by ``delta``."""
    mp = vmap.mean_planes() if mean_planes is None else mean_planes
    return RenderFn.apply(mp, delta, vmap, vmap.grid, cam, poses)
