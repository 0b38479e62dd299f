"""Forward parity of the HIP render kernel against the FP64 oracle (GPU)."""

import zlib

import numpy as np
import pytest
import torch

import scenegen
from scenegen import Camera, Scene, SPEC_BLINN, SPEC_PHONG

from .gpu_common import compare, gpu_render, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2305_07450_amd as rt
    return rt


@pytest.mark.parametrize("seed", [None] + list(range(10)))
def test_workload0_full_frame(rt, oracle_mod, seed):
    """256x144, 8 spheres, 1 light, depth 2: every pixel."""
    wl = scenegen.make_workload(0, seed)
    log("case workload0", wl.scene.digest(), "seed", seed)
    g = gpu_render(rt, wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=True)
    compare(oracle_mod, wl.scene, wl.camera, wl.W, wl.H, wl.depth, g, label=f"w0 seed={seed}",
            **CEILINGS[0])


EDGE_CASES = [
    # (name, W, H, depth, n_spheres, n_lights, plane, spec, camera)
    ("ragged", 37, 23, 2, 6, 1, True, SPEC_BLINN, Camera()),
    ("one_pixel", 1, 1, 3, 5, 1, True, SPEC_BLINN, Camera()),
    ("column", 1, 97, 2, 5, 2, True, SPEC_BLINN, Camera()),
    ("row", 131, 1, 2, 5, 2, True, SPEC_BLINN, Camera()),
    ("portrait", 48, 80, 2, 8, 1, True, SPEC_PHONG, Camera(fov_deg=75.0)),
    ("depth0", 64, 36, 0, 8, 2, True, SPEC_BLINN, Camera()),
    ("depth_max", 64, 36, 8, 12, 2, True, SPEC_BLINN, Camera()),
    ("lights_max", 48, 27, 2, 8, 8, True, SPEC_BLINN, Camera()),
    ("no_lights", 48, 27, 2, 8, 0, True, SPEC_BLINN, Camera()),
    ("no_planes", 64, 36, 3, 10, 1, False, SPEC_PHONG, Camera()),
    ("no_spheres", 64, 36, 2, 0, 1, True, SPEC_BLINN, Camera()),
    ("empty_scene", 16, 9, 2, 0, 1, False, SPEC_BLINN, Camera()),
    ("rotated", 80, 45, 3, 10, 2, True, SPEC_BLINN,
     Camera(eye=(0.5, 0.25, 1.0), yaw_deg=12.0, pitch_deg=-7.5, fov_deg=50.0)),
    ("many_spheres", 72, 40, 2, 300, 2, True, SPEC_BLINN, Camera()),
]


# Ceilings on the ill-conditioned share above the default, measured share
# x ~1.3: eight lights over eight mirror spheres in a 48x27 view put about
# 12 % of the pixels on a shadow edge or a reflected silhouette.
EDGE_CEILINGS = {"lights_max": dict(max_ill=0.15)}


@pytest.mark.parametrize("case", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_cases(rt, oracle_mod, case):
    name, W, H, D, N, L, plane, spec, cam = case
    s = scenegen.tiny_scene(zlib.crc32(name.encode()) % 1000, n_spheres=N, n_lights=L, with_plane=plane,
                            spec_model=spec)
    if name == "no_planes":
        s.background = (0.25, 0.5, 0.75)
        s = Scene(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    log("case", name, W, H, D, N, L)
    g = gpu_render(rt, s, cam, W, H, D, records=True)
    compare(oracle_mod, s, cam, W, H, D, g, label=name, **EDGE_CEILINGS.get(name, {}))


def test_records_do_not_change_image_and_runs_repeat(rt):
    wl = scenegen.make_workload(0, 3)
    a = gpu_render(rt, wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=True)
    b = gpu_render(rt, wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=False)
    c = gpu_render(rt, wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=False)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(b["rgb"], c["rgb"])
    assert np.array_equal(a["ids"], b["ids"])


def test_scene_update_in_place(rt, oracle_mod):
    """rt_scene_update with host and with device arrays gives the image of the new scene."""
    wl = scenegen.make_workload(0, 5)
    s2 = scenegen.perturb_scene(wl.scene, np.random.default_rng(1), sigma=0.2)
    h = rt.SceneHandle(wl.scene)
    try:
        rt.rt_scene_update(h.handle, s2)
        rgb, ids, _ = rt.render(h.handle, wl.camera, wl.W, wl.H, wl.depth, ids=True)
        dev = {k: torch.as_tensor(getattr(s2, k)).cuda() for k in (
            "sphere_geom", "sphere_mat", "sphere_shine", "plane_geom", "plane_mat",
            "plane_shine", "light")}
        keep = rt.rt_scene_update(h.handle, s2, arrays=dev)
        rgb2, ids2, _ = rt.render(h.handle, wl.camera, wl.W, wl.H, wl.depth, ids=True)
        torch.cuda.synchronize()
        del keep
    finally:
        h.close()
    assert torch.equal(rgb, rgb2) and torch.equal(ids, ids2)
    g = dict(rgb=rgb.cpu().numpy().reshape(-1, 3).astype(np.float64),
             ids=ids.cpu().numpy().reshape(-1))
    compare(oracle_mod, s2, wl.camera, wl.W, wl.H, wl.depth, g, label="updated")


# Ceilings per workload: the share of pixels the oracle classifies ill
# conditioned, and the share of non-grazing pixels whose colour is off by more
# than 1e-4 (the mismatch fraction).  Measured values sit well below them
# (see the design notes); a drifting classifier or kernel trips them.
CEILINGS = {0: dict(max_ill=0.04, max_mismatch=0.001),
            1: dict(max_ill=0.12, max_mismatch=0.0005),
            2: dict(max_ill=0.25, max_mismatch=0.005),
            4: dict(max_ill=0.08, max_mismatch=0.0005)}


@pytest.mark.parametrize("config,row_step", [(1, 1), (2, 8), (4, 1)])
def test_full_size_sampled_rows(rt, oracle_mod, config, row_step):
    """Full-size workloads rendered whole on the GPU, in the launch the
    benchmark times; the oracle checks every pixel of a row sample."""
    wl = scenegen.make_workload(config)
    log("case full-size", wl.name, "rows every", row_step)
    g = gpu_render(rt, wl.scene, wl.camera, wl.W, wl.H, wl.depth)
    rows = np.arange(0, wl.H, row_step)
    rows = np.unique(np.concatenate([rows, [wl.H - 1]]))
    pixels = (rows[:, None] * wl.W + np.arange(wl.W)[None, :]).reshape(-1)
    compare(oracle_mod, wl.scene, wl.camera, wl.W, wl.H, wl.depth, g, pixels=pixels,
            label=wl.name, **CEILINGS[config])


@pytest.mark.parametrize("config", [0, 1, 4])
def test_work_counters_match_oracle(rt, oracle_mod, config):
    """The kernel's algorithmic counters equal the oracle's, up to the few
    decisions taken differently at grazing pixels."""
    wl = scenegen.make_workload(config)
    h = rt.SceneHandle(wl.scene)
    try:
        got = rt.render_counts(h.handle, wl.camera, wl.W, wl.H, wl.depth)
    finally:
        h.close()
    want = oracle_mod.render(wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=False,
                             margins=False).counts
    log("counts", wl.name, got, want)
    assert got["primary_rays"] == want["primary_rays"] == wl.W * wl.H
    for k in want:
        assert abs(got[k] - want[k]) <= 1e-3 * max(want[k], 1), (k, got[k], want[k])
    # the culled kernel runs far fewer exact tests than the method counts
    assert 0 < got["exec_sphere_tests"] < got["sphere_tests"]
    assert 0 < got["exec_plane_tests"] <= got["plane_tests"]


@pytest.mark.parametrize("config", [0, 1, 2, 4])
def test_brute_force_kernel_executes_the_method_count(rt, config):
    """Without the cone tests and wave bounds, the kernel executes exactly the
    tests the method counts (every segment every primitive, a shadow ray up
    to its first occluder): executed == algorithmic, bit for bit."""
    wl = scenegen.make_workload(config)
    with rt.SceneHandle(wl.scene) as h:
        c = rt.render_counts(h.handle, wl.camera, wl.W, wl.H, wl.depth,
                             flags=rt.RT_RENDER_NO_PREFILTER)
        culled = rt.render_counts(h.handle, wl.camera, wl.W, wl.H, wl.depth)
    log("brute-force counts", wl.name, c)
    assert c["exec_sphere_tests"] == c["sphere_tests"]
    assert c["exec_plane_tests"] == c["plane_tests"]
    # the culling changes what is executed, not the method's count
    for k in ("sphere_tests", "plane_tests", "primary_rays", "reflection_rays", "shadow_rays"):
        assert c[k] == culled[k], k


ALL_FLAGS = (0, 1)   # with and without the cone prefilters


@pytest.mark.parametrize("config", [0, 1, 2, 4])
def test_prefilters_change_no_bits(rt, config):
    """The cone tests that let a ray skip a sphere (cones seen from the eye
    and from the lights) only skip pairs the exact test rejects: image, ids
    and records are the same bits with them switched off."""
    wl = scenegen.make_workload(config)
    W, H, D = wl.W, wl.H, wl.depth
    with rt.SceneHandle(wl.scene) as h:
        out = []
        for flags in ALL_FLAGS:
            rgb = torch.empty((H, W, 3), device="cuda")
            ids = torch.empty((H, W), dtype=torch.int32, device="cuda")
            rec = rt.Records(W, H, D)
            rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, ids, rec, flags)
            torch.cuda.synchronize()
            out.append((rgb.cpu(), ids.cpu(), rec.buf.cpu()))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert torch.equal(a, b)


@pytest.mark.parametrize("seed", range(6))
def test_prefilters_change_no_bits_small_scenes(rt, seed):
    s = scenegen.tiny_scene(500 + seed, n_spheres=40, n_lights=3, spec_model=seed % 2)
    cam = Camera(eye=(0.3 * seed, 0.5, 0.2), yaw_deg=5.0 * seed - 10.0, pitch_deg=-3.0)
    W, H, D = 123, 77, 5
    with rt.SceneHandle(s) as h:
        imgs = []
        for flags in ALL_FLAGS:
            rgb = torch.empty((H, W, 3), device="cuda")
            rt.rt_render_ex(h.handle, cam, W, H, D, rgb, None, None, flags)
            torch.cuda.synchronize()
            imgs.append(rgb.cpu())
    for im in imgs[1:]:
        assert torch.equal(imgs[0], im)


# Scenes chosen to drive every branch of the wave bounds: several 64-sphere
# chunks with a ragged last one, dense boxes (many sphere-to-sphere mirror
# rays, wide bundles), rotated cameras, ragged image sizes, a light inside a
# sphere and an eye inside a sphere (cones that take every direction).
VARIED = [
    # seed, N, lights, box, W, H, depth, eye, yaw, pitch, light_in, eye_in
    (0, 65, 1, "small", 201, 113, 6, (0.0, 0.0, 0.0), 0.0, 0.0, False, False),
    (1, 100, 2, "wide", 160, 90, 4, (1.0, 1.5, 2.0), 20.0, -10.0, False, False),
    (2, 129, 3, "small", 97, 131, 5, (0.0, 0.3, 0.0), -35.0, 5.0, True, False),
    (3, 200, 4, "wide", 128, 72, 3, (-2.0, 0.0, 1.0), 60.0, 15.0, False, True),
    (4, 300, 2, "small", 150, 100, 8, (0.5, 0.5, -3.0), 170.0, -20.0, True, True),
    (5, 64, 1, "small", 64, 64, 4, (0.0, 5.0, -8.0), 0.0, -89.0, False, False),
]


@pytest.mark.parametrize("case", range(len(VARIED)))
def test_wave_bounds_change_no_bits(rt, case):
    seed, n, L, box, W, H, D, eye, yaw, pitch, light_in, eye_in = VARIED[case]
    rng = np.random.default_rng(900 + seed)
    b = scenegen.BOX_SMALL if box == "small" else ((-20.0, -1.0, -40.0), (20.0, 6.0, -2.0))
    s = scenegen.random_scene(rng, n, L, box=b, spec_model=seed % 2)
    if light_in:
        s.light[0, :3] = s.sphere_geom[0, :3]
    if eye_in:
        eye = tuple(float(v) for v in s.sphere_geom[3, :3])
    cam = Camera(eye=eye, yaw_deg=yaw, pitch_deg=pitch)
    log("case", case, "N", n, "L", L, "size", W, H, "depth", D)
    with rt.SceneHandle(s) as h:
        out = []
        for flags in ALL_FLAGS:
            rgb = torch.empty((H, W, 3), device="cuda")
            ids = torch.empty((H, W), dtype=torch.int32, device="cuda")
            rec = rt.Records(W, H, D)
            rt.rt_render_ex(h.handle, cam, W, H, D, rgb, ids, rec, flags)
            torch.cuda.synchronize()
            out.append((rgb.cpu(), ids.cpu(), rec.buf.cpu()))
    for a, b2 in zip(out[0], out[1]):
        assert torch.equal(a, b2)


def test_wave_bounds_change_no_bits_batch_scenes(rt):
    """All 64 scenes of the batch workload (4 to 1024 spheres in a small box,
    so mirror rays often scatter over every direction): image, ids and
    records are the same bits with and without the bounds."""
    for i, wl in enumerate(scenegen.make_batch()):
        W, H, D = wl.W, wl.H, wl.depth
        log("case batch scene", i, wl.name)
        with rt.SceneHandle(wl.scene) as h:
            out = []
            for flags in ALL_FLAGS:
                rgb = torch.empty((H, W, 3), device="cuda")
                ids = torch.empty((H, W), dtype=torch.int32, device="cuda")
                rec = rt.Records(W, H, D)
                rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, ids, rec, flags)
                torch.cuda.synchronize()
                out.append((rgb.cpu(), ids.cpu(), rec.buf.cpu()))
        for a, b2 in zip(out[0], out[1]):
            assert torch.equal(a, b2), i


@pytest.mark.parametrize("config", [0, 1])
def test_prepared_cones_give_the_same_bits(rt, config):
    """rt_render_prepare followed by rt_render_ex(RT_RENDER_CONES_READY) is
    rt_render split in its two launches: the same image and ids."""
    wl = scenegen.make_workload(config)
    W, H, D = wl.W, wl.H, wl.depth
    with rt.SceneHandle(wl.scene) as h:
        a = torch.empty((H, W, 3), device="cuda")
        ia = torch.empty((H, W), dtype=torch.int32, device="cuda")
        rt.rt_render(h.handle, wl.camera, W, H, D, a, ia)
        # another camera's cones in between, then the prepared render
        other = rt.render(h.handle, Camera(yaw_deg=40.0), W, H, D)
        rt.rt_render_prepare(h.handle, wl.camera, W, H)
        b = torch.empty_like(a)
        ib = torch.empty_like(ia)
        rt.rt_render_ex(h.handle, wl.camera, W, H, D, b, ib, None, rt.RT_RENDER_CONES_READY)
        torch.cuda.synchronize()
        del other
    assert torch.equal(a, b) and torch.equal(ia, ib)


def _render_flags(rt, h, wl, flags, records=False, camera=None):
    """One rt_render_ex into NaN-filled outputs, so that a tile the launch
    skipped cannot pass for a rendered one."""
    W, H, D = wl.W, wl.H, wl.depth
    img = torch.full((H, W, 3), float("nan"), device="cuda")
    ids = torch.full((H, W), -7, dtype=torch.int32, device="cuda")
    rec = rt.Records(W, H, D) if records else None
    rt.rt_render_ex(h.handle, camera or wl.camera, W, H, D, img, ids, rec, flags)
    torch.cuda.synchronize()
    return img, ids, rec


@pytest.mark.parametrize("config", [1, 2, 4])
def test_tile_order_changes_no_bits(rt, config):
    """rt_render records every tile's duration and the next render of the
    scene at that size takes the tiles longest first (1080p, 4K at 129 600
    tiles near the order table's limit, 720p): image, ids and records equal
    the row-order render bit for bit, render after render."""
    wl = scenegen.make_workload(config)
    log("case tile order", wl.name)
    with rt.SceneHandle(wl.scene) as h:
        want, iw, rw = _render_flags(rt, h, wl, rt.RT_RENDER_ROW_ORDER, records=True)
        for k in range(3):   # row order and recording, then two ordered renders
            a, ia, ra = _render_flags(rt, h, wl, 0, records=True)
            assert torch.equal(a, want) and torch.equal(ia, iw), k
            assert torch.equal(ra.ids, rw.ids) and torch.equal(ra.lit, rw.lit), k


def test_tile_order_from_other_views_and_updates(rt):
    """An order measured for another view, after moved spheres, after a
    preparation without a render, and the brute-force variant between
    ordered renders: every image equals the row-order render of its own
    view (1080p workload)."""
    wl = scenegen.make_workload(1)
    W, H, D = wl.W, wl.H, wl.depth
    with rt.SceneHandle(wl.scene) as h:
        for yaw in (0.0, 0.5, 3.0, 20.0, 0.0):
            cam = Camera(yaw_deg=yaw)
            a, ia, _ = _render_flags(rt, h, wl, 0, camera=cam)
            b, ib, _ = _render_flags(rt, h, wl, rt.RT_RENDER_ROW_ORDER, camera=cam)
            assert torch.equal(a, b) and torch.equal(ia, ib), yaw
        s2 = scenegen.random_scene(np.random.default_rng(5), wl.scene.n_spheres, 2,
                                   box=scenegen.BOX_MEDIUM)
        rt.rt_scene_update(h.handle, s2)
        wl2 = scenegen.Workload(wl.name, s2, wl.camera, W, H, D)
        a, ia, _ = _render_flags(rt, h, wl2, 0)
        rt.rt_render_prepare(h.handle, wl.camera, W, H)
        rt.rt_render_prepare(h.handle, wl.camera, W, H)
        c, ic, _ = _render_flags(rt, h, wl2, rt.RT_RENDER_CONES_READY)
        bf, ibf, _ = _render_flags(rt, h, wl2, rt.RT_RENDER_NO_PREFILTER)
        d, id_, _ = _render_flags(rt, h, wl2, 0)
        b, ib, _ = _render_flags(rt, h, wl2, rt.RT_RENDER_ROW_ORDER)
        for x, ix in ((a, ia), (c, ic), (bf, ibf), (d, id_)):
            assert torch.equal(x, b) and torch.equal(ix, ib)


def test_tile_order_of_another_size_is_not_used(rt):
    """A preparation made for one image size leaves rt_render_ex with
    RT_RENDER_CONES_READY at another size in row order: the image equals
    rt_render's at that size (a 720p order table, then a 1080p render, and
    back)."""
    wl = scenegen.make_workload(1)
    D = wl.depth
    with rt.SceneHandle(wl.scene) as h:
        for (W0, H0), (W1, H1) in (((1280, 720), (1920, 1080)), ((1920, 1080), (1280, 720))):
            want = torch.empty((H1, W1, 3), device="cuda")
            rt.rt_render(h.handle, wl.camera, W1, H1, D, want)
            rt.rt_render_prepare(h.handle, wl.camera, W0, H0)
            got = torch.empty_like(want)
            rt.rt_render_ex(h.handle, wl.camera, W1, H1, D, got, None, None,
                            rt.RT_RENDER_CONES_READY)
            torch.cuda.synchronize()
            assert torch.equal(want, got), (W0, H0, W1, H1)


def test_tile_order_with_camera_inside_a_sphere_and_many_planes(rt):
    """Cost estimates of degenerate views: the eye inside a sphere (every
    direction touches it), planes seen from behind and mirror images behind
    their plane; 16 planes x 60 spheres = 1020 entries.  The ordered render
    equals the row-order one."""
    rng = np.random.default_rng(77)
    planes = [(0.0, 1.0, 0.0, -1.0)]
    for k in range(15):
        m = rng.normal(size=3)
        m /= np.linalg.norm(m)
        planes.append((m[0], m[1], m[2], float(rng.uniform(-40.0, 40.0))))
    s = scenegen.random_scene(rng, 60, 2, box=scenegen.BOX_MEDIUM,
                              planes=np.array(planes, dtype=np.float32))
    cam = Camera(eye=tuple(float(v) for v in s.sphere_geom[3, :3]))
    wl = scenegen.Workload("inside", s, cam, 1280, 720, 2)
    with rt.SceneHandle(s) as h:
        a, ia, _ = _render_flags(rt, h, wl, 0)
        b, ib, _ = _render_flags(rt, h, wl, rt.RT_RENDER_ROW_ORDER)
    assert torch.equal(a, b) and torch.equal(ia, ib)


@pytest.mark.parametrize("W,H", [(512, 512), (504, 512), (3072, 3072)])
def test_tile_order_at_the_limits_of_its_range(rt, W, H):
    """The schedule's bounds: 512x512 is exactly 4096 tiles (the smallest
    image ordered), 504x512 one column of tiles fewer (row order, no record),
    3072x3072 147 456 tiles, past the 131 072 the order table holds (row
    order).  Renders after the first equal the row-order render bit for bit
    (NaN-filled outputs), with the bench scene."""
    wl0 = scenegen.make_workload(1)
    wl = scenegen.Workload("limits", wl0.scene, wl0.camera, W, H, 2)
    log("case tile order limits", W, H)
    with rt.SceneHandle(wl.scene) as h:
        want, iw, _ = _render_flags(rt, h, wl, rt.RT_RENDER_ROW_ORDER)
        assert not torch.isnan(want).any()
        for k in range(3):
            a, ia, _ = _render_flags(rt, h, wl, 0)
            assert torch.equal(a, want) and torch.equal(ia, iw), (W, H, k)
