"""Pins of the reference gradient (oracle/grad_ref.py).

The torch re-shade must reproduce the C oracle's image exactly (to FP64
rounding) from the oracle's own records, and its autograd gradient must agree
with central finite differences of the C oracle's masked loss, on pixels whose
decision records do not change under any of the perturbations.  A plain
central difference at h = 1e-3 has an O(h^2) truncation error of up to ~1% on
parameters that move a sharp highlight (exponents up to 64); the pin therefore
uses h = 2.5e-4 refined by one Richardson step with h/2,
(4 D(h/2) - D(h)) / 3, whose error is O(h^4) (measured ~1e-6 relative).
"""

import math

import numpy as np
import pytest

import scenegen
from scenegen import Camera, SPEC_BLINN, SPEC_PHONG

H_FD = 2.5e-4


def _setup(oracle_mod, seed, W=64, H=36, N=8, L=2, D=3, model=SPEC_BLINN):
    rng = np.random.default_rng(seed)
    s = scenegen.random_scene(rng, N, L, spec_model=model)
    base = oracle_mod.render(s, Camera(), W, H, D)
    o, d = oracle_mod.camera_rays(Camera(), W, H, np.arange(W * H))
    return s, base, o, d


@pytest.mark.parametrize("model", [SPEC_BLINN, SPEC_PHONG])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reshade_reproduces_oracle_image(oracle_mod, model, seed):
    from oracle import grad_ref
    s, base, o, d = _setup(oracle_mod, seed, model=model)
    rgb = grad_ref.reshade(grad_ref.params_of(s, False), s, o, d, base.seg_id, base.lit, 3)
    assert np.abs(rgb.numpy() - base.rgb).max() < 1e-12


def _params(s):
    from oracle import grad_ref
    out = []
    for i in range(s.n_spheres):
        out += [("albedo", (i, c)) for c in range(3)]
        out += [("refl", i)]
        out += [("center", (i, c)) for c in range(3)]
    for l in range(s.n_lights):
        out += [("light_pos", (l, c)) for c in range(3)]
        out += [("light_int", l)]
    return out


@pytest.mark.parametrize("model,seed", [(SPEC_BLINN, 3), (SPEC_PHONG, 4), (SPEC_BLINN, 5)])
def test_autograd_matches_central_differences(oracle_mod, model, seed):
    """Every differentiated parameter of a 64x36, 8-sphere, 2-light, depth-3
    scene: autograd of the fixed-visibility re-shade vs central differences of
    the C oracle, on pixels >= 2 px from primary-ID edges whose records stay
    the same at every perturbed point."""
    from oracle import Scene64, grad_ref
    W, H, D = 64, 36, 3
    s, base, o, d = _setup(oracle_mod, seed, W, H, model=model)
    target = scenegen.perturb_scene(s, np.random.default_rng(seed + 99))
    tgt = oracle_mod.render(target, Camera(), W, H, D, records=False, margins=False).rgb
    mask = ~oracle_mod.id_edges(base.prim_id, W, H, radius=2)
    plist = _params(s)
    renders = []
    for name, idx in plist:
        v = grad_ref.get_param(Scene64(s), name, idx)
        pair = []
        for h in (H_FD, H_FD / 2):
            rp = oracle_mod.render(grad_ref.set_param(s, name, idx, v + h), Camera(), W, H, D,
                                   margins=False)
            rm = oracle_mod.render(grad_ref.set_param(s, name, idx, v - h), Camera(), W, H, D,
                                   margins=False)
            for r in (rp, rm):
                mask &= (r.seg_id == base.seg_id).all(1) & (r.lit == base.lit).all(1)
            pair.append((rp.rgb, rm.rgb))
        renders.append(pair)
    assert mask.mean() > 0.4
    loss, grads, rgb = grad_ref.masked_loss_grad(s, o, d, base.seg_id, base.lit, D, tgt, mask)
    m = mask[:, None]
    fd = {k: np.zeros_like(v) for k, v in grads.items()}
    loss_at = lambda rgb: (((rgb - tgt) * m) ** 2).sum()
    for (name, idx), pair in zip(plist, renders):
        d1, d2 = [(loss_at(rp) - loss_at(rm)) / (2 * h)
                  for h, (rp, rm) in zip((H_FD, H_FD / 2), pair)]
        fd[name][idx] = (4 * d2 - d1) / 3
    for k in grads:
        err = np.linalg.norm(fd[k] - grads[k]) / max(np.linalg.norm(fd[k]), 1e-12)
        assert err < 1e-4, (k, err, fd[k].ravel()[:6], grads[k].ravel()[:6])
        assert np.linalg.norm(grads[k]) > 0


def test_lambert_gradient_closed_form(oracle_mod):
    """At the near pole of an on-axis sphere (normal +z, no specular, depth 0):
    dC/dI = a (n.L) and dC/da = k_a + I (n.L)."""
    from oracle import grad_ref
    q = np.array([3.0, 4.0, 2.0])
    s = scenegen.Scene(np.array([[0, 0, -6.0, 1.0]]), np.array([[0.8, 0.5, 0.25, 0.0]]),
                       np.array([16.0]), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                       np.array([[*q, 0.75]]), spec_strength=0.0)
    W, H = 64, 36
    k = np.array([(H // 2) * W + W // 2])
    r = oracle_mod.render(s, Camera(), W, H, 0, pixels=k)
    o, d = oracle_mod.camera_rays(Camera(), W, H, k)
    p = np.array([0.0, 0.0, -5.0])
    nl = (q - p)[2] / np.linalg.norm(q - p)
    a = s.sphere_mat[0, :3].astype(np.float64)
    for c in range(3):
        g = np.zeros((1, 3))
        g[0, c] = 1.0
        grads = grad_ref.vjp(s, o, d, r.seg_id, r.lit, 0, g)
        assert abs(grads["light_int"][0] - a[c] * nl) < 1e-13
        want = np.zeros(3)
        want[c] = float(s.ambient) + 0.75 * nl
        assert np.allclose(grads["albedo"][0], want, atol=1e-13)


def test_directional_derivatives_at_workload4_scale(oracle_mod):
    """Three random directional derivatives of the masked loss for the
    1280x720, 128-sphere, depth-3 workload (every 8th row): autograd of the
    re-shade vs Richardson-refined central differences of the C oracle.

    Kept pixels: well conditioned, records unchanged at every perturbed point,
    and smooth at the step sizes used (per-pixel Richardson estimates from
    steps h and h/2 agree).  Chaotic multi-bounce pixels and segments close to
    a sphere's silhouette have colour derivatives in the hundreds or kinks
    narrower than h; they need far smaller steps.  The filter never looks at
    the analytic gradient."""
    from oracle import Scene64, grad_ref
    prob = scenegen.make_diff_problem()
    wl = prob.workload
    s, W, H, D = wl.scene, wl.W, wl.H, wl.depth
    rows = np.arange(0, H, 8)
    pix = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
    base = oracle_mod.render(s, Camera(), W, H, D, pix)
    tgt = oracle_mod.render(prob.target_scene, Camera(), W, H, D, pix, records=False,
                            margins=False).rgb
    o, d = oracle_mod.camera_rays(Camera(), W, H, pix)
    mask = oracle_mod.condition(s, Camera(), W, H, D, pix, base=base)
    rng = np.random.default_rng(17)
    dirs = [{k: rng.normal(size=v.shape) for k, v in grad_ref.params_of(s, False).items()}
            for _ in range(3)]
    hs = (H_FD / 2, H_FD / 4, H_FD / 8)
    per_dir = []
    for dv in dirs:
        rgb = {}
        for h in hs:
            for sg in (1, -1):
                s2 = Scene64(s)
                hh = sg * h
                s2.sphere_mat[:, :3] += hh * dv["albedo"]
                s2.sphere_mat[:, 3] += hh * dv["refl"]
                s2.sphere_geom[:, :3] += hh * dv["center"]
                s2.light[:, :3] += hh * dv["light_pos"]
                s2.light[:, 3] += hh * dv["light_int"]
                r = oracle_mod.render(s2, Camera(), W, H, D, pix, margins=False)
                mask &= (r.seg_id == base.seg_id).all(1) & (r.lit == base.lit).all(1)
                rgb[hh] = r.rgb
        dc = [(rgb[h] - rgb[-h]) / (2 * h) for h in hs]          # per-pixel dC/dh
        r1 = (4 * dc[1] - dc[0]) / 3
        r2 = (4 * dc[2] - dc[1]) / 3
        mask &= (np.abs(r1 - r2) <= 1e-6 + 1e-4 * np.abs(r2)).all(1)
        per_dir.append(rgb)
    assert mask.mean() > 0.5
    loss, grads, _ = grad_ref.masked_loss_grad(s, o, d, base.seg_id, base.lit, D, tgt, mask)
    m = mask[:, None]
    L = lambda c: (((c - tgt) * m) ** 2).sum()
    for dv, rgb in zip(dirs, per_dir):
        h1, h2 = hs[0], hs[1]
        d1 = (L(rgb[h1]) - L(rgb[-h1])) / (2 * h1)
        d2 = (L(rgb[h2]) - L(rgb[-h2])) / (2 * h2)
        fd = (4 * d2 - d1) / 3
        an = sum(float((grads[k] * dv[k]).sum()) for k in grads)
        assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-12), (fd, an)


@pytest.mark.parametrize("model,seed", [(SPEC_BLINN, 0), (SPEC_PHONG, 1)])
def test_reshade_reproduces_oracle_image_with_sky(oracle_mod, model, seed):
    from oracle import grad_ref
    rng = np.random.default_rng(seed)
    s = scenegen.random_scene(rng, 8, 2, spec_model=model)
    sky = scenegen.sky_map(seed=seed, w=96, h=48).astype(np.float64)
    W, H, D = 64, 36, 3
    base = oracle_mod.render(s, Camera(), W, H, D, sky=sky)
    o, d = oracle_mod.camera_rays(Camera(), W, H, np.arange(W * H))
    rgb = grad_ref.reshade(grad_ref.params_of(s, False), s, o, d, base.seg_id, base.lit, D, sky)
    assert (base.seg_id == -1).any()
    assert np.abs(rgb.numpy() - base.rgb).max() < 1e-12


def test_autograd_through_the_sky_matches_central_differences(oracle_mod):
    """Every differentiated parameter with a skybox: autograd of the re-shade
    (through the UV mapping and the bilinear weights of the misses) vs
    Richardson-refined central differences of the C oracle.  Kept pixels: the
    records stay the same at every perturbed point, and the per-pixel
    estimates from steps h and h/2 agree (the bilinear colour has a kink at
    every texel boundary, which a step may cross)."""
    from oracle import Scene64, grad_ref
    W, H, D = 64, 36, 3
    rng = np.random.default_rng(8)
    s = scenegen.random_scene(rng, 8, 2)
    sky = scenegen.sky_map(seed=9, w=48, h=24).astype(np.float64)
    cam = Camera(pitch_deg=8.0)
    base = oracle_mod.render(s, cam, W, H, D, sky=sky)
    o, d = oracle_mod.camera_rays(cam, W, H, np.arange(W * H))
    target = scenegen.perturb_scene(s, np.random.default_rng(108))
    tgt = oracle_mod.render(target, cam, W, H, D, records=False, margins=False, sky=sky).rgb
    mask = ~oracle_mod.id_edges(base.prim_id, W, H, radius=2)
    plist = _params(s)
    hs = (H_FD, H_FD / 2, H_FD / 4)
    renders = []
    for name, idx in plist:
        v = grad_ref.get_param(Scene64(s), name, idx)
        rgb = {}
        for h in hs:
            for sg in (1, -1):
                r = oracle_mod.render(grad_ref.set_param(s, name, idx, v + sg * h), cam, W, H, D,
                                      margins=False, sky=sky)
                mask &= (r.seg_id == base.seg_id).all(1) & (r.lit == base.lit).all(1)
                rgb[sg * h] = r.rgb
        dc = [(rgb[h] - rgb[-h]) / (2 * h) for h in hs]
        r1, r2 = (4 * dc[1] - dc[0]) / 3, (4 * dc[2] - dc[1]) / 3
        mask &= (np.abs(r1 - r2) <= 1e-6 + 1e-4 * np.abs(r2)).all(1)
        renders.append(rgb)
    assert mask.mean() > 0.4
    # misses after a bounce carry the sky's gradient into the sphere centres
    reflected_miss = (base.seg_id[:, 0] >= 0) & (base.seg_id == -1).any(1) & mask
    assert reflected_miss.sum() > 20
    loss, grads, _ = grad_ref.masked_loss_grad(s, o, d, base.seg_id, base.lit, D, tgt, mask, sky)
    m = mask[:, None]
    loss_at = lambda rgb: (((rgb - tgt) * m) ** 2).sum()
    fd = {k: np.zeros_like(v) for k, v in grads.items()}
    for (name, idx), rgb in zip(plist, renders):
        d1, d2 = [(loss_at(rgb[h]) - loss_at(rgb[-h])) / (2 * h) for h in hs[:2]]
        fd[name][idx] = (4 * d2 - d1) / 3
    for k in grads:
        err = np.linalg.norm(fd[k] - grads[k]) / max(np.linalg.norm(fd[k]), 1e-12)
        assert err < 1e-4, (k, err)
    # the sky term matters: without it the centre gradient is different
    no_sky = grad_ref.masked_loss_grad(s, o, d, base.seg_id, base.lit, D, tgt, mask)[1]
    assert np.linalg.norm(no_sky["center"] - grads["center"]) > 1e-3 * np.linalg.norm(
        grads["center"])
