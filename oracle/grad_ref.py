"""Reference gradients of the rendered image with visibility held fixed.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper defines no derivative; the differentiated quantity is the image of
the Whitted tracer (Sections 3.3-3.7) as a function of the continuous scene
parameters, with every discrete decision frozen: the primitive hit by each
segment, the set of lights that light each hit (n.L > 0 and no occluder), and
the depth at which the path ends.  Those decisions come from the C oracle's
per-segment records.  This module re-shades each path from its records in
torch float64 on the CPU and lets autograd differentiate it.

It is written in the front-to-back form (throughput T starting at 1, colour C
accumulated per segment) instead of the C oracle's recursion; the two agree
exactly in real arithmetic, which ``tests/test_oracle_grad.py`` checks to
rounding, and central finite differences of the C oracle pin the gradient.

Differentiated parameters: sphere albedo [N,3], sphere reflection ratio [N],
sphere centre [N,3], light position [L,3], light intensity [L].  Radii,
exponents, planes, ambient and k_s are constants; shadow occluders carry no
gradient.  With a skybox (Section 3.8) a path that ends in a miss adds T times
the map's bilinear colour in the ray's direction, written out as the C oracle
computes it; its texels are constants, and autograd differentiates through
the UV mapping and the bilinear weights (the texel indices are decisions).
"""

from __future__ import annotations

import math
from typing import Dict

import numpy as np
import torch

from scenegen import Scene, SPEC_PHONG

PARAM_NAMES = ("albedo", "refl", "center", "light_pos", "light_int")


def params_of(scene: Scene, requires_grad: bool = True) -> Dict[str, torch.Tensor]:
    f = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=requires_grad)
    return dict(albedo=f(scene.sphere_mat[:, :3]), refl=f(scene.sphere_mat[:, 3]),
                center=f(scene.sphere_geom[:, :3]), light_pos=f(scene.light[:, :3]),
                light_int=f(scene.light[:, 3]))


def _dot(a, b):
    return (a * b).sum(-1)


def _sky(sky: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """Bilinear skybox colour [n,3] in directions d [n,3]: u = 1/2 +
    atan2(d_x, -d_z)/(2 pi), v = 1/2 - asin(d_y)/pi, texel centres at
    x = u w - 1/2, y = v h - 1/2, wrapping in x and clamping in y."""
    h, w = sky.shape[0], sky.shape[1]
    u = 0.5 + torch.atan2(d[:, 0], -d[:, 2]) / (2.0 * math.pi)
    v = 0.5 - torch.asin(torch.clamp(d[:, 1], -1.0, 1.0)) / math.pi
    x = u * w - 0.5
    y = v * h - 0.5
    fx, fy = torch.floor(x.detach()), torch.floor(y.detach())
    ax, ay = (x - fx)[:, None], (y - fy)[:, None]
    x0, y0 = fx.long(), fy.long()
    xs = [torch.remainder(x0 + k, w) for k in (0, 1)]
    ys = [torch.clamp(y0 + k, 0, h - 1) for k in (0, 1)]
    t = lambda yi, xi: sky[yi, xi]
    return ((1.0 - ay) * ((1.0 - ax) * t(ys[0], xs[0]) + ax * t(ys[0], xs[1]))
            + ay * ((1.0 - ax) * t(ys[1], xs[0]) + ax * t(ys[1], xs[1])))


def reshade(params: Dict[str, torch.Tensor], scene: Scene, o0: np.ndarray, d0: np.ndarray,
            seg_id: np.ndarray, lit: np.ndarray, depth: int, sky=None) -> torch.Tensor:
    """Colour [n,3] of n paths with fixed records (seg_id, lit: [n, depth+1]);
    `sky` is the skybox [h, w, 3] or None for the plain background."""
    dt = torch.float64
    N, P, L = scene.n_spheres, scene.n_planes, scene.n_lights
    radius = torch.tensor(scene.sphere_geom[:, 3], dtype=dt)
    shine = torch.tensor(np.concatenate([scene.sphere_shine, scene.plane_shine]), dtype=dt)
    pgeom = torch.tensor(scene.plane_geom, dtype=dt)
    palb = torch.tensor(scene.plane_mat[:, :3], dtype=dt)
    pkr = torch.tensor(scene.plane_mat[:, 3], dtype=dt)
    bg = torch.tensor(scene.background, dtype=dt)
    sky_t = torch.tensor(np.asarray(sky, dtype=np.float64)) if sky is not None else None
    ka, ks, tmin = float(scene.ambient), float(scene.spec_strength), float(scene.t_min)
    albedo = torch.cat([params["albedo"], palb], 0)         # [N+P, 3]
    kr_all = torch.cat([params["refl"], pkr], 0)            # [N+P]
    seg = torch.as_tensor(seg_id.astype(np.int64))
    litm = torch.as_tensor(lit.astype(np.int64))
    n_pix = seg.shape[0]
    o = torch.tensor(o0, dtype=dt)
    d = torch.tensor(d0, dtype=dt)
    T = torch.ones(n_pix, dtype=dt)
    C = torch.zeros(n_pix, 3, dtype=dt)
    alive = torch.ones(n_pix, dtype=torch.bool)
    for k in range(depth + 1):
        idk = seg[:, k]
        miss = alive & (idk == -1)
        if sky_t is not None and bool(miss.any()):
            C = C + torch.where(miss[:, None], T[:, None] * _sky(sky_t, d), torch.zeros_like(C))
        else:
            C = C + torch.where(miss[:, None], T[:, None] * bg, torch.zeros_like(C))
        hit = alive & (idk >= 0)
        if not bool(hit.any()):
            break
        ids = torch.where(hit, idk, torch.zeros_like(idk))
        sph = hit & (ids < N)
        pl = hit & (ids >= N)
        si = torch.where(sph, ids, torch.zeros_like(ids)).clamp(max=max(N - 1, 0))
        pj = torch.where(pl, ids - N, torch.zeros_like(ids)).clamp(min=0, max=max(P - 1, 0))
        # hit distance of the recorded primitive: sphere root (near root above
        # t_min, else the far root) or plane root
        if N:
            c = params["center"][si]
            r = radius[si]
            oc = o - c
            b = _dot(oc, d)
            q = _dot(oc, oc) - r * r
            disc = torch.where(sph, b * b - q, torch.ones_like(b))
            sq = torch.sqrt(torch.clamp(disc, min=1e-300))
            t_near, t_far = -b - sq, -b + sq
            t_s = torch.where(t_near > tmin, t_near, t_far)
        else:
            c = torch.zeros_like(o)
            r = torch.ones(n_pix, dtype=dt)
            t_s = torch.ones(n_pix, dtype=dt)
        if P:
            m = pgeom[pj, :3]
            h = pgeom[pj, 3]
            den = _dot(m, d)
            den = torch.where(pl, den, torch.ones_like(den))
            t_p = (h - _dot(m, o)) / den
        else:
            m = torch.zeros_like(o)
            t_p = torch.ones(n_pix, dtype=dt)
        t = torch.where(sph, t_s, torch.where(pl, t_p, torch.ones_like(t_s)))
        p = o + t[:, None] * d
        n_s = (p - c) / r[:, None]
        n = torch.where(sph[:, None], n_s, m)
        view = -d
        A = torch.full((n_pix,), ka, dtype=dt)
        S = torch.zeros(n_pix, dtype=dt)
        sh = shine[ids]
        for l in range(L):
            bit = hit & (((litm[:, k] >> l) & 1) == 1)
            if not bool(bit.any()):
                continue
            lv = params["light_pos"][l] - p
            ld = lv / torch.sqrt(_dot(lv, lv))[:, None]
            nl = _dot(n, ld)
            I = params["light_int"][l]
            if scene.spec_model == SPEC_PHONG:
                rv = 2.0 * nl[:, None] * n - ld
                x = _dot(view, rv)
            else:
                hv = ld + view
                x = _dot(n, hv) / torch.sqrt(torch.clamp(_dot(hv, hv), min=1e-300))
            xs = torch.where(bit & (x > 0), x, torch.ones_like(x))
            spec = torch.where(bit & (x > 0), torch.pow(xs, sh), torch.zeros_like(x))
            A = A + torch.where(bit, I * nl, torch.zeros_like(nl))
            S = S + torch.where(bit, I * ks * spec, torch.zeros_like(spec))
        a = albedo[ids]
        kr = kr_all[ids]
        if k < depth:
            contrib = T[:, None] * (A[:, None] * (1.0 - kr)[:, None] * a + S[:, None])
            C = C + torch.where(hit[:, None], contrib, torch.zeros_like(C))
            T = torch.where(hit, T * A * kr, T)
            dn = _dot(d, n)
            d_new = d - 2.0 * dn[:, None] * n
            o = torch.where(hit[:, None], p, o)
            d = torch.where(hit[:, None], d_new, d)
        else:
            contrib = T[:, None] * (A[:, None] * a + S[:, None])
            C = C + torch.where(hit[:, None], contrib, torch.zeros_like(C))
        alive = hit
    return C


def masked_loss_grad(scene: Scene, o0, d0, seg_id, lit, depth, target_rgb: np.ndarray,
                     mask: np.ndarray, sky=None):
    """Loss = sum over masked pixels of |C - target|^2; returns (loss, grads,
    rgb) with grads a dict of float64 numpy arrays keyed by PARAM_NAMES."""
    prm = params_of(scene)
    C = reshade(prm, scene, o0, d0, seg_id, lit, depth, sky)
    diff = (C - torch.tensor(target_rgb, dtype=torch.float64)) * torch.tensor(
        mask.astype(np.float64))[:, None]
    loss = (diff * diff).sum()
    loss.backward()
    return float(loss.detach()), _grads(prm), C.detach().numpy()


def vjp(scene: Scene, o0, d0, seg_id, lit, depth, grad_rgb: np.ndarray, sky=None):
    """Gradient of sum(grad_rgb * C) with respect to every parameter group."""
    prm = params_of(scene)
    C = reshade(prm, scene, o0, d0, seg_id, lit, depth, sky)
    (C * torch.tensor(grad_rgb, dtype=torch.float64)).sum().backward()
    return _grads(prm)


def _grads(prm):
    return {k: (prm[k].grad.detach().numpy().copy() if prm[k].grad is not None
                else np.zeros(tuple(prm[k].shape))) for k in PARAM_NAMES}


def set_param(scene, name: str, index, value: float):
    """FP64 copy (oracle.Scene64) of a scene with one scalar parameter replaced."""
    from oracle import Scene64
    s = Scene64(scene)
    arr, sl = _locate(s, name, index)
    arr[sl] = value
    return s


def get_param(scene, name: str, index) -> float:
    arr, sl = _locate(scene, name, index)
    return float(arr[sl])


def _locate(s, name: str, index):
    i = index
    if name == "albedo":
        return s.sphere_mat, (i[0], i[1])
    if name == "refl":
        return s.sphere_mat, (i, 3)
    if name == "center":
        return s.sphere_geom, (i[0], i[1])
    if name == "light_pos":
        return s.light, (i[0], i[1])
    if name == "light_int":
        return s.light, (i, 3)
    raise KeyError(name)
