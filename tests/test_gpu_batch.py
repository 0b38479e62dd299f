"""Batched persistent launch (rt_batch_*) on the GPU.

Every image of a batch must be bit-identical to a single rt_render of the
same scene (same per-pixel code), for the graph replay and the direct launch,
for autotuned and default launch shapes, on every replay."""

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


def small_batch():
    out = []
    specs = [(64, 36, 2, 5, 1), (37, 23, 0, 3, 2), (1, 1, 3, 4, 1), (130, 70, 4, 40, 1),
             (16, 100, 1, 9, 3), (96, 54, 3, 0, 1)]
    for i, (W, H, D, N, L) in enumerate(specs):
        s = scenegen.tiny_scene(40 + i, n_spheres=N, n_lights=L, spec_model=i % 2)
        cam = Camera(yaw_deg=float(i - 2), fov_deg=55.0 + i)
        out.append(scenegen.Workload(f"b{i}", s, cam, W, H, D))
    return out


def single_images(rt, wls, handles):
    imgs = []
    for wl, h in zip(wls, handles):
        rgb = torch.empty((wl.H, wl.W, 3), device="cuda")
        rt.rt_render(h.handle, wl.camera, wl.W, wl.H, wl.depth, rgb)
        imgs.append(rgb)
    torch.cuda.synchronize()
    return [im.cpu() for im in imgs]


def make_batch(rt, wls, handles, autotune):
    outs = [torch.full((wl.H, wl.W, 3), float("nan"), device="cuda") for wl in wls]
    b = rt.rt_batch_create([h.handle for h in handles], [w.camera for w in wls],
                           [w.W for w in wls], [w.H for w in wls], [w.depth for w in wls], outs,
                           autotune=autotune)
    return b, outs


@pytest.mark.parametrize("autotune", [False, True])
def test_small_batch_bit_exact(rt, autotune):
    wls = small_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        ref = single_images(rt, wls, handles)
        b, outs = make_batch(rt, wls, handles, autotune)
        try:
            log("batch shape", rt.rt_batch_shape(b))
            for rep in range(3):
                for o in outs:
                    o.fill_(float("nan"))
                if rep == 1:
                    rt.rt_batch_launch_direct(b)
                else:
                    rt.rt_batch_launch(b)
                torch.cuda.synchronize()
                for i, (o, r) in enumerate(zip(outs, ref)):
                    assert torch.equal(o.cpu(), r), (rep, i)
                # eager work between replays
                torch.randn(1000, device="cuda").sum().item()
        finally:
            rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()


def test_autotune_cache_persists_the_timed_shape(rt, tmp_path, monkeypatch):
    """A tuned batch stores its shape under its key in the JSON file; another
    process reads it; a new batch of the same signature takes the stored
    shape instead of timing (a planted shape shows which), with the same
    images."""
    import json
    import os
    import subprocess
    import sys
    monkeypatch.setenv("RT_TUNE_CACHE", str(tmp_path / "tune.json"))
    rt.rt_tune_cache_forget()
    wls = small_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        ref = single_images(rt, wls, handles)
        b, outs = make_batch(rt, wls, handles, True)
        key, shape = rt.rt_batch_tune_key(b), rt.rt_batch_shape(b)
        rt.rt_batch_destroy(b)
        arch = torch.cuda.get_device_properties(0).gcnArchName
        log("tuned", shape, "key", key[:80])
        assert key.startswith(arch + ":")
        assert rt.rt_tune_cache_get(key) == shape
        code = ("import sys, paper_2305_07450_amd as rt; "
                "print(rt.rt_tune_cache_get(sys.argv[1]))")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        child = subprocess.run([sys.executable, "-c", code, key], cwd=root, env=dict(os.environ),
                               capture_output=True, text=True, timeout=300)
        assert child.returncode == 0, child.stderr
        assert child.stdout.strip().splitlines()[-1] == str(shape)
        planted = (96, 64, 4) if shape != (96, 64, 4) else (160, 8, 16)
        rt.rt_tune_cache_put(key, *planted)
        rt.rt_tune_cache_forget()
        assert len(json.load(open(tmp_path / "tune.json"))["entries"]) == 1
        b, outs = make_batch(rt, wls, handles, True)
        try:
            assert rt.rt_batch_shape(b) == planted
            rt.rt_batch_launch(b)
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ref)):
                assert torch.equal(o.cpu(), r), i
        finally:
            rt.rt_batch_destroy(b)
    finally:
        rt.rt_tune_cache_forget()
        for h in handles:
            h.close()


def test_batch_image_matches_oracle(rt, oracle_mod):
    wls = small_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        b, outs = make_batch(rt, wls, handles, False)
        rt.rt_batch_launch(b)
        torch.cuda.synchronize()
        wl = wls[3]
        ids = torch.empty((wl.H, wl.W), dtype=torch.int32, device="cuda")
        rgb = torch.empty((wl.H, wl.W, 3), device="cuda")
        rt.rt_render(handles[3].handle, wl.camera, wl.W, wl.H, wl.depth, rgb, ids)
        torch.cuda.synchronize()
        g = dict(rgb=outs[3].cpu().numpy().reshape(-1, 3).astype(np.float64),
                 ids=ids.cpu().numpy().reshape(-1))
        compare(oracle_mod, wl.scene, wl.camera, wl.W, wl.H, wl.depth, g, label="batch image 3")
        rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()


# The four densest scenes of the 64-scene batch (about 900 spheres in the small
# box): index, rows sampled every `step`.
DENSE_BATCH_SCENES = ((18, 16), (3, 16), (8, 16), (40, 1))


def test_workload3_densest_scenes_match_oracle(rt, oracle_mod):
    """The batch's own output for its densest scenes, where brute force is
    costliest (about 900 spheres), against the FP64 oracle on sampled rows;
    primary ids come from a single render, which the batch equals bit for bit."""
    wls = scenegen.make_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        b, outs = make_batch(rt, wls, handles, True)
        rt.rt_batch_launch(b)
        torch.cuda.synchronize()
        for i, step in DENSE_BATCH_SCENES:
            wl = wls[i]
            log("case batch scene", i, wl.name, "spheres", wl.scene.n_spheres)
            ids = torch.empty((wl.H, wl.W), dtype=torch.int32, device="cuda")
            rgb = torch.empty((wl.H, wl.W, 3), device="cuda")
            rt.rt_render(handles[i].handle, wl.camera, wl.W, wl.H, wl.depth, rgb, ids)
            torch.cuda.synchronize()
            assert torch.equal(rgb, outs[i])
            g = dict(rgb=outs[i].cpu().numpy().reshape(-1, 3).astype(np.float64),
                     ids=ids.cpu().numpy().reshape(-1))
            rows = np.unique(np.concatenate([np.arange(0, wl.H, step), [wl.H - 1]]))
            pixels = (rows[:, None] * wl.W + np.arange(wl.W)[None, :]).reshape(-1)
            compare(oracle_mod, wl.scene, wl.camera, wl.W, wl.H, wl.depth, g, pixels=pixels,
                    label=f"batch dense {i}", max_ill=0.30, max_mismatch=0.01)
        rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()


def test_scene_update_between_replays(rt):
    wls = small_batch()[:3]
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        b, outs = make_batch(rt, wls, handles, False)
        rt.rt_batch_launch(b)
        torch.cuda.synchronize()
        first = outs[0].cpu()
        s2 = scenegen.perturb_scene(wls[0].scene, np.random.default_rng(0), sigma=0.3)
        rt.rt_scene_update(handles[0].handle, s2)
        rt.rt_batch_launch(b)
        torch.cuda.synchronize()
        assert not torch.equal(outs[0].cpu(), first)
        ref = torch.empty_like(outs[0])
        rt.rt_render(handles[0].handle, wls[0].camera, wls[0].W, wls[0].H, wls[0].depth, ref)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], ref)
        rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()


def test_workload3_64_scenes(rt):
    """The 64-scene batch workload: every image equals its single render."""
    wls = scenegen.make_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    try:
        ref = single_images(rt, wls, handles)
        b, outs = make_batch(rt, wls, handles, True)
        log("batch shape", rt.rt_batch_shape(b))
        rt.rt_batch_launch(b)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o.cpu(), r), i
        rt.rt_batch_destroy(b)
    finally:
        for h in handles:
            h.close()


def test_batch_rejects_bad_arguments(rt):
    wl = small_batch()[0]
    with rt.SceneHandle(wl.scene) as h:
        out = torch.empty((wl.H, wl.W, 3), device="cuda")
        with pytest.raises(rt.RtError):
            rt.rt_batch_create([h.handle], [wl.camera], [wl.W], [wl.H], [9], [out])
        with pytest.raises(rt.RtError):
            rt.rt_batch_create([h.handle], [Camera(fov_deg=0.0)], [wl.W], [wl.H], [1], [out])
        with pytest.raises(rt.RtError):
            rt.rt_batch_create([], [], [], [], [], [])
