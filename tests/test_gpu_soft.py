"""Soft shadows on the GPU (rt_render_soft), against the FP64 oracle.

Parity bar as for hard shadows (tests/gpu_common.py): primary ids bit-exact
off grazing pixels and colour within 1e-4 on pixels the oracle's jittered
re-traces classify as well conditioned.  Every sample ray moves with its
segment in those re-traces, so a pixel whose visible-sample count is
sensitive to rounding shows a colour spread and is set aside; the share set
aside is reported.  The wave bounds only skip spheres the exact test
rejects, so the image is the same bits with them switched off."""

import numpy as np
import pytest
import torch

import scenegen
from scenegen import Camera

from .gpu_common import compare, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2305_07450_amd as rt
    return rt


def soft_render(rt, scene, cam, W, H, D, samples, radius, flags=0):
    with rt.SceneHandle(scene) as h:
        rgb = torch.empty((H, W, 3), device="cuda")
        ids = torch.empty((H, W), dtype=torch.int32, device="cuda")
        rt.rt_render_soft(h.handle, cam, W, H, D, samples, radius, rgb, ids, flags)
        torch.cuda.synchronize()
        return dict(rgb=rgb.cpu().numpy().reshape(-1, 3).astype(np.float64),
                    ids=ids.cpu().numpy().reshape(-1))


@pytest.mark.parametrize("seed", range(4))
def test_soft_parity_small_scenes(rt, oracle_mod, seed):
    s = scenegen.tiny_scene(700 + seed, n_spheres=10, n_lights=2, spec_model=seed % 2)
    cam = Camera(yaw_deg=3.0 * seed - 4.0, pitch_deg=-4.0)
    W, H, D, n, R = 96, 54, 2, 32, 0.6
    log("case soft small", seed, W, H, D, n, R)
    g = soft_render(rt, s, cam, W, H, D, n, R)
    stats, base = compare(oracle_mod, s, cam, W, H, D, g, label=f"soft{seed}", samples=n,
                          light_radius=R)
    # the penumbrae are in the image: some pixel sees part of a light
    assert (stats["ill_conditioned"] < 0.25), stats


def test_soft_parity_paper_scene(rt, oracle_mod):
    s = scenegen.paper_scene()
    cam = Camera()
    W, H = 192, 108
    n, D = scenegen.PAPER_SETTINGS["soft200_3bounces"]
    R = scenegen.PAPER_LIGHT_RADIUS
    log("case soft paper scene", W, H, D, n, R)
    g = soft_render(rt, s, cam, W, H, D, n, R)
    compare(oracle_mod, s, cam, W, H, D, g, label="soft_paper", samples=n, light_radius=R)


SOFT_BITS = [
    # (scene kind, N, lights, W, H, depth, samples, radius)
    ("paper", 5, 1, 320, 180, 3, 200, 0.5),
    ("small", 40, 2, 123, 77, 4, 64, 0.8),
    ("small", 100, 3, 96, 60, 3, 50, 0.4),      # two chunks of spheres
    ("small", 300, 1, 80, 50, 2, 24, 0.6),      # beyond the bounded chunks: full scans
    ("bench", 64, 2, 480, 270, 4, 200, 0.5),
]


@pytest.mark.parametrize("case", range(len(SOFT_BITS)))
def test_soft_bounds_change_no_bits(rt, case):
    kind, N, L, W, H, D, n, R = SOFT_BITS[case]
    if kind == "paper":
        s = scenegen.paper_scene()
    elif kind == "bench":
        s = scenegen.make_workload(1).scene
    else:
        s = scenegen.random_scene(np.random.default_rng(810 + case), N, L)
    cam = Camera(yaw_deg=2.0, pitch_deg=-3.0)
    log("case soft bits", case, kind, N, L, W, H, D, n, R)
    a = soft_render(rt, s, cam, W, H, D, n, R, 0)
    b = soft_render(rt, s, cam, W, H, D, n, R, rt.RT_RENDER_NO_PREFILTER)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["ids"], b["ids"])


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


# Planes that the sample rays of whole waves can be shown not to reach are not
# tested for them; these scenes put lights, spheres and planes near the edges
# of that proof: lights just above or below the floor, spheres through it,
# a wall behind the spheres and a tilted plane.
PLANE_CASES = [
    ("low lights", ((-4.0, -1.5, -12.0), (4.0, 1.0, -4.0)), ((-5.0, -0.95, -10.0), (5.0, -0.2, -2.0)),
     scenegen.GROUND),
    ("floor and wall", scenegen.BOX_SMALL, scenegen.LIGHT_BOX,
     np.array([[0.0, 1.0, 0.0, -1.0], [0.0, 0.0, 1.0, -14.0]], dtype=np.float32)),
    ("tilted plane", scenegen.BOX_SMALL, scenegen.LIGHT_BOX,
     np.array([[*_unit([0.3, 0.9, 0.1]), -1.5]], dtype=np.float32)),
    ("lights under the floor", scenegen.BOX_SMALL, ((-5.0, -4.0, -10.0), (5.0, -1.2, -2.0)),
     scenegen.GROUND),
]


@pytest.mark.parametrize("case", range(len(PLANE_CASES)))
def test_soft_plane_skip_changes_no_bits(rt, case):
    label, box, light_box, planes = PLANE_CASES[case]
    s = scenegen.random_scene(np.random.default_rng(930 + case), 24, 2, box=box,
                              light_box=light_box, planes=planes)
    cam = Camera(pitch_deg=-6.0)
    W, H, D, n, R = 112, 64, 3, 64, 0.8
    log("case soft plane skip", label, W, H, D, n, R)
    a = soft_render(rt, s, cam, W, H, D, n, R, 0)
    b = soft_render(rt, s, cam, W, H, D, n, R, rt.RT_RENDER_NO_PREFILTER)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["ids"], b["ids"]), label


# Images of up to 40 000 tiles share each pixel's samples between two lanes;
# larger ones give each pixel one lane.  Both sides of that limit, with and
# without the bounds and skips (the same bits either way).
@pytest.mark.parametrize("W,H", [(1600, 1600), (1608, 1600)])
def test_soft_lanes_per_pixel_limit_changes_no_bits(rt, W, H):
    s = scenegen.paper_scene()
    cam = Camera(yaw_deg=4.0, pitch_deg=-2.0)
    D, n, R = 2, 24, scenegen.PAPER_LIGHT_RADIUS
    log("case soft lanes per pixel", W, H, D, n, R)
    a = soft_render(rt, s, cam, W, H, D, n, R, 0)
    b = soft_render(rt, s, cam, W, H, D, n, R, rt.RT_RENDER_NO_PREFILTER)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["ids"], b["ids"])


def test_one_sample_or_radius_zero_is_point_light(rt):
    s = scenegen.tiny_scene(71, n_spheres=20, n_lights=2)
    cam = Camera(pitch_deg=-5.0)
    W, H, D = 77, 45, 3
    with rt.SceneHandle(s) as h:
        ref = torch.empty((H, W, 3), device="cuda")
        rt.rt_render(h.handle, cam, W, H, D, ref)
        for n, R in ((1, 0.7), (16, 0.0)):
            img = torch.empty((H, W, 3), device="cuda")
            rt.rt_render_soft(h.handle, cam, W, H, D, n, R, img)
            torch.cuda.synchronize()
            assert torch.equal(img, ref), (n, R)


def test_soft_shadows_change_shading_not_visibility(rt):
    """An area light changes the shading (penumbrae) but not what the
    primary rays hit."""
    s = scenegen.paper_scene()
    cam = Camera()
    W, H, D = 160, 90, 1
    a = soft_render(rt, s, cam, W, H, D, 1, 0.0)
    b = soft_render(rt, s, cam, W, H, D, 100, 0.5)
    assert not np.array_equal(a["rgb"], b["rgb"])
    assert np.array_equal(a["ids"], b["ids"])


def test_soft_rejects_bad_arguments(rt):
    s = scenegen.tiny_scene(3)
    with rt.SceneHandle(s) as h:
        out = torch.empty((10, 10, 3), device="cuda")
        for n, R in ((0, 0.5), (rt.RT_MAX_SAMPLES + 1, 0.5), (8, -1.0), (8, float("nan")),
                     (8, float("inf"))):
            with pytest.raises(rt.RtError):
                rt.rt_render_soft(h.handle, Camera(), 10, 10, 1, n, R, out)
        with pytest.raises(rt.RtError):
            rt.rt_render_soft(h.handle, Camera(), 10, 10, 1, 8, 0.5, out, None, 8)


def test_soft_tile_order_changes_no_bits(rt):
    """rt_render_soft records its tiles' durations and the next soft render of
    the scene at that size takes the tiles longest first; hard-shadow renders
    in between record for themselves.  Every image equals the row-order soft
    render bit for bit (bench scene, 1280x720, 14 400 tiles)."""
    s = scenegen.make_workload(1).scene
    cam = Camera(yaw_deg=1.0)
    W, H, D, n, R = 1280, 720, 3, 48, 0.5
    log("case soft tile order", W, H, D, n, R)

    def soft(h, flags):
        img = torch.full((H, W, 3), float("nan"), device="cuda")
        ids = torch.full((H, W), -7, dtype=torch.int32, device="cuda")
        rt.rt_render_soft(h.handle, cam, W, H, D, n, R, img, ids, flags)
        torch.cuda.synchronize()
        return img, ids

    with rt.SceneHandle(s) as h:
        want, iw = soft(h, rt.RT_RENDER_ROW_ORDER)
        hard = torch.empty((H, W, 3), device="cuda")
        for k in range(5):   # records, ordered, ordered; a hard render; again
            if k == 3:
                rt.rt_render(h.handle, cam, W, H, D, hard)
            a, ia = soft(h, 0)
            assert torch.equal(a, want) and torch.equal(ia, iw), k
        bf, ibf = soft(h, rt.RT_RENDER_NO_PREFILTER)
        assert torch.equal(bf, want) and torch.equal(ibf, iw)
