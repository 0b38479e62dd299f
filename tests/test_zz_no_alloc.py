"""rt_render_backward_static, the adjoint entry point that allocates nothing,
against rt_render_backward (GPU, through the C ABI).

Both calls run the same kernels on the same grid; only the buffer of the
per-workgroup partials differs (a file-scope device array instead of the
scene's buffer), so the gradients must agree bit for bit.  Two problems in a
row, the second smaller, show that rows left over from a larger call are
never read; a problem whose partials exceed the array is refused before any
launch.
"""

import numpy as np
import pytest
import torch

import scenegen
from scenegen import Camera

from .gpu_common import log

pytestmark = pytest.mark.gpu

GROUPS = ("albedo", "refl", "center", "light_pos", "light_int")


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2305_07450_amd as rt
    return rt


def _grads(scene):
    N, L = scene.n_spheres, scene.n_lights
    shapes = dict(albedo=(N, 3), refl=(N,), center=(N, 3), light_pos=(L, 3), light_int=(L,))
    return {k: torch.full(s, float("nan"), device="cuda") for k, s in shapes.items()}


def _both(rt, scene, cam, W, H, D, seed):
    """Gradients of one random dLoss/dRGB from both entry points, with records
    and re-traced."""
    g_np = np.random.default_rng(seed).normal(size=(H, W, 3)).astype(np.float32)
    grad_rgb = torch.tensor(g_np, device="cuda")
    out = {}
    with rt.SceneHandle(scene) as h:
        _, _, rec = rt.render(h.handle, cam, W, H, D, ids=False, records=True)
        for mode, r in (("checkpoint", rec), ("recompute", None)):
            for name, fn in (("static", rt.rt_render_backward_static),
                             ("scene", rt.rt_render_backward)):
                g = _grads(scene)
                fn(h.handle, cam, W, H, D, grad_rgb, g, r)
                torch.cuda.synchronize()
                out[(mode, name)] = {k: v.cpu().numpy() for k, v in g.items()}
    return out


def test_static_scratch_matches_scene_partials_two_calls(rt):
    prob = scenegen.make_diff_problem()
    wl = prob.workload
    small = scenegen.tiny_scene(31, n_spheres=9, n_lights=2)
    cases = [(wl.scene, wl.camera, wl.W, wl.H, wl.depth, "workload 4"),
             (small, Camera(), 40, 23, 3, "small")]
    for i, (scene, cam, W, H, D, label) in enumerate(cases):
        log("case no-alloc backward", label, W, H, D, scene.n_spheres, scene.n_lights)
        out = _both(rt, scene, cam, W, H, D, seed=100 + i)
        for mode in ("checkpoint", "recompute"):
            a, b = out[(mode, "static")], out[(mode, "scene")]
            for k in GROUPS:
                assert np.isfinite(a[k]).all(), (label, mode, k)
                assert np.array_equal(a[k], b[k]), (label, mode, k,
                                                    float(np.abs(a[k] - b[k]).max()))
        assert all(np.array_equal(out[("checkpoint", "static")][k],
                                  out[("recompute", "static")][k]) for k in GROUPS)


def test_static_scratch_refuses_oversized_partials(rt):
    """4096 spheres and 8 lights over a 512x512 image need 584 partial rows of
    28704 floats (67 MB), beyond the 16 MiB array: refused, nothing written."""
    s = scenegen.random_scene(np.random.default_rng(7), rt.RT_MAX_SPHERES, rt.RT_MAX_LIGHTS,
                              box=scenegen.BOX_LARGE, radii=scenegen.RADII_SMALL)
    W, H, D = 512, 512, 1
    log("case no-alloc refusal", W, H, D, s.n_spheres)
    with rt.SceneHandle(s) as h:
        g = _grads(s)
        grad_rgb = torch.ones((H, W, 3), device="cuda")
        with pytest.raises(rt.RtError) as e:
            rt.rt_render_backward_static(h.handle, Camera(), W, H, D, grad_rgb, g, None)
        assert e.value.status == rt.RT_ERR_INVALID_ARG
        assert "static scratch" in str(e.value)
        torch.cuda.synchronize()
        assert all(bool(torch.isnan(v).all()) for v in g.values()), "refused call wrote"
