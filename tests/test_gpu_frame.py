"""The interactive per-frame path (rt_frame_*) on the GPU.

Every frame streams a camera, the bounce limit (and the soft-shadow
samples) and new sphere centres in, and the image out, through a replayed
HIP graph whose node parameters change per frame.  Each replay is checked
bit for bit against the eager path on a second copy of the scene:
rt_scene_update with the same centres, then rt_render_ex / rt_render_soft.
The centres come from a Verlet integration of the paper-scene stand-in (the
paper's physics system moves its bodies that way), the camera orbits.  One
frame is also checked against the FP64 oracle."""

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


def moved(scene, pos):
    s = scene.copy()
    s.sphere_geom = s.sphere_geom.copy()
    s.sphere_geom[:, :3] = pos
    return s


def orbit(k):
    return Camera(eye=(0.1 * k, 0.3, 0.0), yaw_deg=-6.0 + 1.5 * k, pitch_deg=-5.0 + 0.5 * k)


def eager(rt, h, scene_k, cam, W, H, D, soft, n, R):
    rt.rt_scene_update(h.handle, scene_k)
    img = torch.empty((H, W, 3), device="cuda")
    if soft:
        rt.rt_render_soft(h.handle, cam, W, H, D, n, R, img)
    else:
        rt.rt_render_ex(h.handle, cam, W, H, D, img)
    torch.cuda.synchronize()
    return img.cpu()


@pytest.mark.parametrize("soft,sky,stream_out", [(False, False, True), (True, False, False),
                                                 (False, True, False), (True, True, True)])
def test_frames_equal_eager_renders(rt, soft, sky, stream_out):
    s = scenegen.paper_scene()
    W, H = 160, 90
    n_frames = 10
    motion = scenegen.verlet_motion(s, n_frames)
    n, D = scenegen.PAPER_SETTINGS["soft200_3bounces" if soft else "hard_1bounce"]
    R = scenegen.PAPER_LIGHT_RADIUS if soft else 0.0
    n = n if soft else 1
    log("case frames", soft, sky, stream_out)
    sky_map = scenegen.sky_map(w=128, h=64) if sky else None
    out = torch.full((H, W, 3), float("nan"), device="cuda")
    with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
        if sky:
            rt.rt_scene_set_sky(hf.handle, sky_map)
            rt.rt_scene_set_sky(he.handle, sky_map)
        f = rt.rt_frame_create(hf.handle, W, H, out, soft=soft, stream_out=stream_out)
        try:
            for k in range(n_frames):
                cam = orbit(k)
                depth = D + (k % 2)                   # the bounce limit changes too
                rt.rt_frame_submit(f, cam, depth, n, R, motion[k])
                host = rt.rt_frame_result(f, W, H)
                got = out.cpu()
                want = eager(rt, he, moved(s, motion[k]), cam, W, H, depth, soft, n, R)
                assert torch.equal(got, want), k
                if stream_out:
                    assert np.array_equal(host, want.numpy()), k
                else:
                    assert host is None
        finally:
            rt.rt_frame_destroy(f)


def test_pipelined_frames_keep_their_images(rt):
    """Frame k+1 is submitted before frame k is taken: results come back in
    order, and each host image stays intact until the second submit after
    its own."""
    s = scenegen.paper_scene()
    W, H, D = 128, 72, 1
    motion = scenegen.verlet_motion(s, 6, seed=3)
    out = torch.empty((H, W, 3), device="cuda")
    with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
        want = [eager(rt, he, moved(s, motion[k]), orbit(k), W, H, D, False, 1, 0.0).numpy()
                for k in range(6)]
        f = rt.rt_frame_create(hf.handle, W, H, out, stream_out=True)
        try:
            rt.rt_frame_submit(f, orbit(0), D, 1, 0.0, motion[0])
            for k in range(1, 6):
                rt.rt_frame_submit(f, orbit(k), D, 1, 0.0, motion[k])
                img = rt.rt_frame_result(f, W, H)          # frame k - 1
                assert np.array_equal(img, want[k - 1]), k
            assert np.array_equal(rt.rt_frame_result(f, W, H), want[5])
            with pytest.raises(rt.RtError):
                rt.rt_frame_result(f, W, H)                # none waiting
            # three submits without taking any: the oldest is dropped
            for k in range(3):
                rt.rt_frame_submit(f, orbit(k), D, 1, 0.0, motion[k])
            assert np.array_equal(rt.rt_frame_result(f, W, H), want[1])
            assert np.array_equal(rt.rt_frame_result(f, W, H), want[2])
        finally:
            rt.rt_frame_destroy(f)


def argb8(img):
    """The packed pixel format, written from its definition: each channel
    floor(clamp(c, 0, 1) * 255 + 0.5) in FP32, alpha 255 on top."""
    x = np.clip(np.asarray(img, np.float32), np.float32(0), np.float32(1))
    q = np.floor(x * np.float32(255) + np.float32(0.5)).astype(np.uint32)
    return (np.uint32(0xFF000000) | (q[..., 0] << 16) | (q[..., 1] << 8) | q[..., 2])


@pytest.mark.parametrize("soft,pipelined", [(False, True), (True, True), (False, False)])
def test_packed_pixels_stream_out(rt, soft, pipelined):
    """Packed 32-bit pixels streamed out, with frame k+1 submitted before
    frame k is taken (pipelined) or each frame taken at once: every frame's
    pixels equal the packing of the eager float image, and the device float
    image is the eager image."""
    s = scenegen.paper_scene()
    W, H = 150, 83
    motion = scenegen.verlet_motion(s, 7, seed=5)
    n, D = scenegen.PAPER_SETTINGS["soft200_3bounces" if soft else "hard_1bounce"]
    n = n if soft else 1
    R = scenegen.PAPER_LIGHT_RADIUS if soft else 0.0
    out = torch.empty((H, W, 3), device="cuda")
    with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
        sky = scenegen.sky_map(w=96, h=48)
        rt.rt_scene_set_sky(hf.handle, sky)
        rt.rt_scene_set_sky(he.handle, sky)
        want = [eager(rt, he, moved(s, motion[k]), orbit(k), W, H, D, soft, n, R)
                for k in range(7)]
        assert any(((w.numpy() > 1) | (w.numpy() < 0)).any() for w in want)  # clamping is used
        f = rt.rt_frame_create(hf.handle, W, H, out, soft=soft, stream_out=True,
                               fmt=rt.RT_FRAME_ARGB8)
        try:
            if pipelined:
                rt.rt_frame_submit(f, orbit(0), D, n, R, motion[0])
                for k in range(1, 7):
                    rt.rt_frame_submit(f, orbit(k), D, n, R, motion[k])
                    px = rt.rt_frame_result(f, W, H, rt.RT_FRAME_ARGB8)    # frame k - 1
                    assert px.dtype == np.uint32 and px.shape == (H, W)
                    assert np.array_equal(px, argb8(want[k - 1].numpy())), k
            else:
                for k in range(6):
                    rt.rt_frame_submit(f, orbit(k), D, n, R, motion[k])
                    px = rt.rt_frame_result(f, W, H, rt.RT_FRAME_ARGB8)    # frame k
                    assert np.array_equal(px, argb8(want[k].numpy())), k
                rt.rt_frame_submit(f, orbit(6), D, n, R, motion[6])
            px = rt.rt_frame_result(f, W, H, rt.RT_FRAME_ARGB8)
            assert np.array_equal(px, argb8(want[6].numpy()))
            assert torch.equal(out.cpu(), want[6])
            # a skybox removed between frames rebuilds the graphs
            rt.rt_scene_set_sky(hf.handle, None)
            rt.rt_scene_set_sky(he.handle, None)
            rt.rt_frame_submit(f, orbit(6), D, n, R, None)
            px = rt.rt_frame_result(f, W, H, rt.RT_FRAME_ARGB8)
            ref = eager(rt, he, moved(s, motion[6]), orbit(6), W, H, D, soft, n, R)
            assert np.array_equal(px, argb8(ref.numpy()))
        finally:
            rt.rt_frame_destroy(f)


def test_frame_matches_oracle(rt, oracle_mod):
    s = scenegen.paper_scene()
    W, H = 192, 108
    motion = scenegen.verlet_motion(s, 30)
    k = 29
    cam = orbit(k)
    out = torch.empty((H, W, 3), device="cuda")
    with rt.SceneHandle(s) as h:
        f = rt.rt_frame_create(h.handle, W, H, out)
        try:
            for j in range(k + 1):
                rt.rt_frame_submit(f, orbit(j), 1, 1, 0.0, motion[j])
            rt.rt_frame_result(f)
            rt.rt_frame_result(f)
        finally:
            rt.rt_frame_destroy(f)
    g = dict(rgb=out.cpu().numpy().reshape(-1, 3).astype(np.float64),
             ids=np.zeros(W * H, np.int32))
    sk = moved(s, motion[k])
    base = oracle_mod.render(sk, cam, W, H, 1)
    g["ids"] = base.prim_id.copy()      # the frame path writes no ids: colour only
    compare(oracle_mod, sk, cam, W, H, 1, g, label="frame29")


def test_kept_positions_scene_updates_and_sky_toggle(rt):
    """NULL positions keep the spheres where they are; an rt_scene_update
    between frames (new materials) and a skybox added or removed between
    frames are seen by the next frame."""
    s = scenegen.paper_scene()
    W, H, D = 96, 64, 2
    motion = scenegen.verlet_motion(s, 3, seed=11)
    out = torch.empty((H, W, 3), device="cuda")
    cam = orbit(4)
    with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
        f = rt.rt_frame_create(hf.handle, W, H, out)
        try:
            rt.rt_frame_submit(f, cam, D, 1, 0.0, motion[2])
            rt.rt_frame_result(f)
            rt.rt_frame_submit(f, cam, D, 1, 0.0, None)
            rt.rt_frame_result(f)
            s2 = moved(s, motion[2])
            assert torch.equal(out.cpu(), eager(rt, he, s2, cam, W, H, D, False, 1, 0.0))
            s3 = s2.copy()
            s3.sphere_mat = s3.sphere_mat.copy()
            s3.sphere_mat[:, :3] = s3.sphere_mat[:, ::-1][:, 1:4]
            rt.rt_scene_update(hf.handle, s3)
            rt.rt_frame_submit(f, cam, D, 1, 0.0, None)
            rt.rt_frame_result(f)
            assert torch.equal(out.cpu(), eager(rt, he, s3, cam, W, H, D, False, 1, 0.0))
            sky = scenegen.sky_map(w=64, h=32)
            rt.rt_scene_set_sky(hf.handle, sky)
            rt.rt_scene_set_sky(he.handle, sky)
            rt.rt_frame_submit(f, cam, D, 1, 0.0, None)
            rt.rt_frame_result(f)
            assert torch.equal(out.cpu(), eager(rt, he, s3, cam, W, H, D, False, 1, 0.0))
            rt.rt_scene_set_sky(hf.handle, None)
            rt.rt_scene_set_sky(he.handle, None)
            rt.rt_frame_submit(f, cam, D, 1, 0.0, None)
            rt.rt_frame_result(f)
            assert torch.equal(out.cpu(), eager(rt, he, s3, cam, W, H, D, False, 1, 0.0))
        finally:
            rt.rt_frame_destroy(f)


def test_frame_rejects_bad_inputs(rt):
    s = scenegen.paper_scene()
    out = torch.empty((8, 8, 3), device="cuda")
    with rt.SceneHandle(s) as h:
        hard = rt.rt_frame_create(h.handle, 8, 8, out)
        soft = rt.rt_frame_create(h.handle, 8, 8, out, soft=True)
        try:
            bad_pos = scenegen.verlet_motion(s, 1)[0].copy()
            bad_pos[2, 1] = np.nan
            for f, args in ((hard, (1, 2, 0.5, None)), (soft, (1, 1, 0.5, None)),
                            (soft, (1, 8, 0.0, None)), (soft, (1, 8, float("inf"), None)),
                            (soft, (1, rt.RT_MAX_SAMPLES + 1, 0.5, None)),
                            (hard, (9, 1, 0.0, None)), (hard, (-1, 1, 0.0, None)),
                            (hard, (1, 1, 0.0, bad_pos))):
                with pytest.raises(rt.RtError) as e:
                    rt.rt_frame_submit(f, Camera(), *args)
                assert e.value.status == rt.RT_ERR_INVALID_ARG
            with pytest.raises(rt.RtError):
                rt.rt_frame_submit(hard, Camera(fov_deg=200.0), 1, 1, 0.0, None)
            with pytest.raises(rt.RtError):
                rt.rt_frame_result(hard)                    # nothing submitted
        finally:
            rt.rt_frame_destroy(hard)
            rt.rt_frame_destroy(soft)


def test_frames_of_small_and_empty_scenes(rt):
    """A 1x1 image, a scene without spheres (no positions to stream) and a
    scene without lights run through the frame path as through the eager
    one."""
    cases = [("one pixel", scenegen.paper_scene(), 1, 1),
             ("no spheres", scenegen.tiny_scene(3, n_spheres=0, n_lights=2), 33, 17),
             ("no lights", scenegen.tiny_scene(4, n_spheres=7, n_lights=0), 29, 31)]
    for name, s, W, H in cases:
        log("case frame", name)
        out = torch.empty((H, W, 3), device="cuda")
        pos = scenegen.verlet_motion(s, 3, seed=2)
        with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
            f = rt.rt_frame_create(hf.handle, W, H, out, stream_out=True, fmt=rt.RT_FRAME_ARGB8)
            try:
                for k in range(3):
                    rt.rt_frame_submit(f, orbit(k), 2, 1, 0.0, pos[k] if pos.shape[1] else None)
                    px = rt.rt_frame_result(f, W, H, rt.RT_FRAME_ARGB8)
                    want = eager(rt, he, moved(s, pos[k]), orbit(k), W, H, 2, False, 1, 0.0)
                    assert torch.equal(out.cpu(), want), (name, k)
                    assert np.array_equal(px, argb8(want.numpy())), (name, k)
            finally:
                rt.rt_frame_destroy(f)


@pytest.mark.parametrize("soft", [False, True])
def test_frames_without_prefilters(rt, soft):
    """A frame object made with RT_RENDER_NO_PREFILTER renders what the eager
    calls render with that flag, which is also the image with the bounds."""
    s = scenegen.paper_scene()
    W, H = 96, 54
    motion = scenegen.verlet_motion(s, 3, seed=4)
    n, D = scenegen.PAPER_SETTINGS["soft200_3bounces" if soft else "hard_1bounce"]
    n = n if soft else 1
    R = scenegen.PAPER_LIGHT_RADIUS if soft else 0.0
    out = torch.empty((H, W, 3), device="cuda")
    with rt.SceneHandle(s) as hf, rt.SceneHandle(s) as he:
        f = rt.rt_frame_create(hf.handle, W, H, out, soft=soft, flags=rt.RT_RENDER_NO_PREFILTER)
        try:
            for k in range(3):
                rt.rt_frame_submit(f, orbit(k), D, n, R, motion[k])
                rt.rt_frame_result(f)
                got = out.cpu()
                rt.rt_scene_update(he.handle, moved(s, motion[k]))
                ref = torch.empty((H, W, 3), device="cuda")
                for flags in (rt.RT_RENDER_NO_PREFILTER, 0):
                    if soft:
                        rt.rt_render_soft(he.handle, orbit(k), W, H, D, n, R, ref, None, flags)
                    else:
                        rt.rt_render_ex(he.handle, orbit(k), W, H, D, ref, None, None, flags)
                    torch.cuda.synchronize()
                    assert torch.equal(got, ref.cpu()), (k, flags)
        finally:
            rt.rt_frame_destroy(f)
