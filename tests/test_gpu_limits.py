"""The library's declared limits on the GPU, against the FP64 oracle.

  * a scene at RT_MAX_SPHERES spheres, RT_MAX_PLANES planes and RT_MAX_LIGHTS
    lights (64 chunks of spheres behind every wave bound);
  * images RT_MAX_DIM pixels wide and RT_MAX_DIM pixels tall;
  * RT_MAX_SAMPLES shadow samples per light;
  * soft shadows in a scene past the sphere chunks the soft bound covers, so
    every sample ray scans every sphere;
  * the adjoint at RT_MAX_SPHERES spheres (its accumulators take 112 KiB of
    LDS, within the 160 KiB a gfx950 workgroup may hold);
  * a batch of RT_MAX_BATCH scenes.

The parity bar is the one of the other forward tests (tests/gpu_common.py);
the batch is compared bit for bit with single renders."""

import numpy as np
import pytest
import torch

import scenegen
from scenegen import Camera

from .gpu_common import compare, gpu_render, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2305_07450_amd as rt
    return rt


def sixteen_planes() -> np.ndarray:
    """The ground, a ceiling and four walls around the sphere box, and ten
    tilted planes 60 to 120 units out, every normal facing the origin."""
    walls = np.array([[0, 1, 0, -1], [0, -1, 0, -40], [1, 0, 0, -45], [-1, 0, 0, -45],
                      [0, 0, 1, -150], [0, 0, -1, -40]], dtype=np.float64)
    rng = np.random.default_rng(1616)
    m = rng.normal(size=(10, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    tilted = np.concatenate([m, -rng.uniform(60.0, 120.0, size=(10, 1))], axis=1)
    return np.concatenate([walls, tilted]).astype(np.float32)


def max_scene(rt, n_spheres=None):
    planes = sixteen_planes()
    assert planes.shape[0] == rt.RT_MAX_PLANES
    return scenegen.random_scene(np.random.default_rng(4096),
                                 n_spheres or rt.RT_MAX_SPHERES, rt.RT_MAX_LIGHTS,
                                 box=scenegen.BOX_LARGE, radii=scenegen.RADII_SMALL,
                                 planes=planes, intensity=0.25)


def test_largest_scene(rt, oracle_mod):
    s = max_scene(rt)
    cam = Camera(eye=(0.0, 1.0, 0.0), pitch_deg=-4.0)
    W, H, D = 48, 27, 2
    log("case limits scene", s.n_spheres, "spheres", s.plane_geom.shape[0], "planes",
        s.n_lights, "lights", W, H, D)
    g = gpu_render(rt, s, cam, W, H, D, records=True)
    # 4096 spheres of radius 0.1-0.6 in a 48x27 view: about 39 % of the
    # pixels sit on a silhouette, shadow edge or reflected edge
    stats, base = compare(oracle_mod, s, cam, W, H, D, g, label="max_scene", max_ill=0.45)
    # the view is crowded: about half the primary rays hit a sphere
    assert (base.prim_id < s.n_spheres).mean() > 0.4, stats


@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_largest_image_side(rt, oracle_mod, shape):
    wl = scenegen.make_workload(1)
    W, H = (rt.RT_MAX_DIM, 2) if shape == "wide" else (2, rt.RT_MAX_DIM)
    # the field of view spans the short side: 0.02 degrees over 2 pixels
    # opens the long side to about 55 degrees either way
    cam = Camera(fov_deg=0.02, pitch_deg=-3.0)
    D = 2
    log("case limits image", W, H, D)
    g = gpu_render(rt, wl.scene, cam, W, H, D)
    # a 0.02 degree short side: a pixel row spans the whole scene, so about
    # 15 % of the wide image's pixels straddle an edge
    compare(oracle_mod, wl.scene, cam, W, H, D, g, label=f"max_dim_{shape}", max_ill=0.18)


def soft_render(rt, scene, cam, W, H, D, samples, radius):
    with rt.SceneHandle(scene) as h:
        rgb = torch.empty((H, W, 3), device="cuda")
        ids = torch.empty((H, W), dtype=torch.int32, device="cuda")
        rt.rt_render_soft(h.handle, cam, W, H, D, samples, radius, rgb, ids, 0)
        torch.cuda.synchronize()
        return dict(rgb=rgb.cpu().numpy().reshape(-1, 3).astype(np.float64),
                    ids=ids.cpu().numpy().reshape(-1))


def test_most_shadow_samples(rt, oracle_mod):
    s = scenegen.paper_scene()
    cam = Camera()
    W, H, D, n, R = 32, 18, 1, rt.RT_MAX_SAMPLES, scenegen.PAPER_LIGHT_RADIUS
    log("case limits samples", W, H, D, n, R)
    g = soft_render(rt, s, cam, W, H, D, n, R)
    compare(oracle_mod, s, cam, W, H, D, g, label="max_samples", samples=n, light_radius=R)


def test_soft_shadows_past_the_bounded_chunks(rt, oracle_mod):
    """400 spheres: more than the four 64-sphere chunks the soft bound
    keeps candidate masks for, so every sample ray tests every sphere."""
    s = scenegen.random_scene(np.random.default_rng(400), 400, 2, box=scenegen.BOX_MEDIUM,
                              radii=scenegen.RADII_SMALL)
    cam = Camera(pitch_deg=-5.0)
    W, H, D, n, R = 64, 36, 2, 16, 0.5
    log("case limits soft scan", s.n_spheres, W, H, D, n, R)
    g = soft_render(rt, s, cam, W, H, D, n, R)
    # 400 small spheres, 16 samples per light: about 16 % of the pixels see
    # a sample ray graze an occluder
    compare(oracle_mod, s, cam, W, H, D, g, label="soft_scan", samples=n, light_radius=R,
            max_ill=0.20)


def test_adjoint_at_the_sphere_limit(rt, oracle_mod):
    from .test_gpu_backward import reference_check
    s = max_scene(rt)
    assert s.n_spheres == rt.RT_MAX_SPHERES
    target = scenegen.perturb_scene(s, np.random.default_rng(2336))
    cam = Camera(eye=(0.0, 1.0, 0.0), pitch_deg=-4.0)
    W, H, D = 48, 27, 2
    log("case limits adjoint", s.n_spheres, W, H, D)
    reference_check(rt, oracle_mod, s, cam, W, H, D, target, "adjoint_max")


def test_largest_batch(rt):
    """RT_MAX_BATCH jobs over four scenes, ragged tiny images of depths
    0 to 3: every image equals the single render, for the graph replay and
    the direct launch."""
    n = rt.RT_MAX_BATCH
    handles = [rt.SceneHandle(scenegen.tiny_scene(60 + i, n_spheres=3 + 5 * i, n_lights=1 + i % 2))
               for i in range(4)]
    try:
        jobs = []
        for j in range(n):
            W, H = 3 + j % 11, 2 + (j // 11) % 7
            cam = Camera(yaw_deg=float(j % 37) - 18.0, pitch_deg=float(j % 13) - 6.0)
            jobs.append((handles[j % 4], cam, W, H, j % 4))
        log("case limits batch", n, "jobs")
        ref = []
        for h, cam, W, H, D in jobs:
            rgb = torch.empty((H, W, 3), device="cuda")
            rt.rt_render(h.handle, cam, W, H, D, rgb)
            ref.append(rgb)
        outs = [torch.full((H, W, 3), float("nan"), device="cuda") for _, _, W, H, _ in jobs]
        b = rt.rt_batch_create([h.handle for h, *_ in jobs], [c for _, c, *_ in jobs],
                               [W for _, _, W, _, _ in jobs], [H for _, _, _, H, _ in jobs],
                               [D for *_, D in jobs], outs, autotune=False)
        try:
            for launch in (rt.rt_batch_launch, rt.rt_batch_launch_direct):
                for o in outs:
                    o.fill_(float("nan"))
                launch(b)
                torch.cuda.synchronize()
                got = torch.cat([o.reshape(-1) for o in outs]).cpu()
                want = torch.cat([r.reshape(-1) for r in ref]).cpu()
                assert torch.equal(got, want), launch.__name__
        finally:
            rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()
