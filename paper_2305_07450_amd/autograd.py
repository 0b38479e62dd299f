"""torch.autograd wrapper around rt_render / rt_render_backward.

The forward pass writes the scene's differentiated parameters into the
uploaded scene (rt_scene_update with device arrays) and renders; when the
records of every segment fit the budget (RT_RECORD_BUDGET_BYTES, default
4 GiB) they are kept for the backward pass ("checkpoint"), otherwise the
adjoint kernel re-traces the decisions itself ("recompute").  Both modes give
bit-identical gradients.
"""

from __future__ import annotations

import os
from typing import Optional

import torch

from . import (Records, rt_records_bytes, rt_render, rt_render_backward, rt_scene_update)

DEFAULT_BUDGET = 4 << 30


def record_budget() -> int:
    return int(os.environ.get("RT_RECORD_BUDGET_BYTES", DEFAULT_BUDGET))


class FixedParts:
    """Scene parts that are not differentiated, on the device: radius [N],
    sphere exponent [N], planes, constants."""

    def __init__(self, scene, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        self.radius = f(scene.sphere_geom[:, 3])
        self.sphere_shine = f(scene.sphere_shine)
        self.plane_geom = f(scene.plane_geom).reshape(-1, 4)
        self.plane_mat = f(scene.plane_mat).reshape(-1, 4)
        self.plane_shine = f(scene.plane_shine).reshape(-1)
        self.ambient = scene.ambient
        self.spec_strength = scene.spec_strength
        self.t_min = scene.t_min
        self.background = scene.background
        self.spec_model = scene.spec_model


def _arrays(albedo, refl, center, light_pos, light_int, fixed: FixedParts):
    return dict(
        sphere_geom=torch.cat([center, fixed.radius[:, None]], 1).contiguous(),
        sphere_mat=torch.cat([albedo, refl[:, None]], 1).contiguous(),
        sphere_shine=fixed.sphere_shine,
        plane_geom=fixed.plane_geom, plane_mat=fixed.plane_mat, plane_shine=fixed.plane_shine,
        light=torch.cat([light_pos, light_int[:, None]], 1).contiguous())


class RTRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, albedo, refl, center, light_pos, light_int, fixed, handle, camera, W, H,
                depth, mode):
        arrays = _arrays(albedo.detach(), refl.detach(), center.detach(), light_pos.detach(),
                         light_int.detach(), fixed)
        rt_scene_update(handle, fixed, arrays=arrays)
        keep = mode == "checkpoint" and rt_records_bytes(W, H, depth) <= record_budget()
        rec = Records(W, H, depth, albedo.device) if keep else None
        rgb = torch.empty((H, W, 3), dtype=torch.float32, device=albedo.device)
        rt_render(handle, camera, W, H, depth, rgb, None, rec)
        ctx.arrays = arrays
        ctx.rec = rec
        ctx.args = (fixed, handle, camera, W, H, depth)
        ctx.shapes = (albedo.shape, refl.shape, center.shape, light_pos.shape, light_int.shape)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        fixed, handle, camera, W, H, depth = ctx.args
        # the scene may have been updated since the forward pass
        rt_scene_update(handle, fixed, arrays=ctx.arrays)
        dev = grad_rgb.device
        grads = {k: torch.empty(s, dtype=torch.float32, device=dev) for k, s in zip(
            ("albedo", "refl", "center", "light_pos", "light_int"), ctx.shapes)}
        rt_render_backward(handle, camera, W, H, depth, grad_rgb.contiguous().float(), grads,
                           ctx.rec)
        return (grads["albedo"], grads["refl"], grads["center"], grads["light_pos"],
                grads["light_int"], None, None, None, None, None, None, None)


def render_differentiable(albedo, refl, center, light_pos, light_int, fixed: FixedParts,
                          handle: int, camera, W: int, H: int, depth: int,
                          mode: str = "checkpoint"):
    """Image [H, W, 3] as a differentiable function of sphere albedo [N,3],
    reflection ratio [N], centre [N,3], light position [L,3] and intensity [L]."""
    if mode not in ("checkpoint", "recompute"):
        raise ValueError("mode must be 'checkpoint' or 'recompute'")
    return RTRender.apply(albedo, refl, center, light_pos, light_int, fixed, handle, camera, W,
                          H, depth, mode)
