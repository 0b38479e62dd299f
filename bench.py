#!/usr/bin/env python3
"""Benchmark of the Whitted render kernel on one MI355X.

A step is one rt_render of the 1920x1080 workload (64 spheres + ground plane,
2 point lights, reflection depth 4, one primary ray per pixel, seeded
synthetic scene): the preparation launch (eye cones, tile order), then the
render kernel (primary rays, closest hits, shading with shadow rays and the
mirror bounces of every pixel).  The scene is resident in HBM before timing
starts; the image stays in HBM.  The render takes its tiles longest first by
the durations the previous render of the scene at this size measured; the
JSON also gives the row-order loop, the first render of a fresh upload and a
turning camera.

The timed region is exactly --steps rt_render calls with nothing between
them; ms_per_step is the larger of its HIP-event and host wall-clock means.
Prints one JSON line: primary Mrays/s (value), fps, total Mrays/s, the frame
time distribution (mean, median, the paper's mean of 10 consecutive frames,
from a second loop with one event between frames),
the FP32 ALU roofline of the render kernel from the exact tests it executes,
the brute-force variant (no culling) with its own fraction, the batched and
forward+backward workloads, and the FP64 CPU oracle timed on the host beside
the parity statistics of the headline frame.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3         # MI355X vector FP32 (packed), 256 CU x 256 FLOP/clk x 2.4 GHz
FLOP_SPHERE_TEST = 16            # oc 3, b 5, |oc|^2 5, -r^2 1, b^2 - q 2 (FMA = 2)
FLOP_PLANE_TEST = 12             # m.d 5, h - m.o 6, divide 1


def test_flops(counts, executed: bool) -> int:
    """FLOPs of the ray-primitive tests: the ones the kernel executed, or the
    method's algorithmic count (every segment every primitive)."""
    if executed:
        return (FLOP_SPHERE_TEST * counts["exec_sphere_tests"]
                + FLOP_PLANE_TEST * counts["exec_plane_tests"])
    return FLOP_SPHERE_TEST * counts["sphere_tests"] + FLOP_PLANE_TEST * counts["plane_tests"]


def frac_of_peak(flops: float, ms: float) -> float:
    return flops / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS


def executed_fp32(prof: dict, ms: float):
    """All FP32 arithmetic the render kernel issues (rocprofv3 VALU counts x
    lane utilisation, from the committed profile of this kernel source), per
    launch and as a rate over `ms`; None when the source has changed."""
    f = prof.get("executed_fp32_flops_per_launch")
    if not f:
        return None
    return {"flops_per_launch": f, "tflops": round(f / (ms * 1e-3) / 1e12, 3),
            "frac": round(frac_of_peak(f, ms), 4),
            "source": "(2 x FMA_F32 + ADD_F32 + MUL_F32) x 64 x lane utilisation, "
                      "profiles/render_traffic.json"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_traffic.json")
ADJOINT_FILE = os.path.join(ROOT, "profiles", "adjoint_fp32.json")
CSRC = "paper_2305_07450_amd/csrc/"
KERNEL_SOURCES = (CSRC + "trace.hpp", CSRC + "render.hip")
ADJOINT_SOURCES = (CSRC + "trace.hpp", CSRC + "adjoint.hip")


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_digest() -> str:
    return source_digest(KERNEL_SOURCES)


def measured_profile(path: str, sources, workload: str) -> dict:
    """Figures per launch from a committed rocprofv3 counter run (HBM bytes,
    FP32 instruction counts), or {} when the kernel source has changed since
    they were taken."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_digest") != source_digest(sources) or t.get("workload") != workload:
        return {}
    return t


def frame_parity(oracle, wl, gpu_rgb, gpu_ids, threads):
    """Parity of the headline frame against the FP64 oracle, the bar of the
    GPU parity tests: primary ids on non-grazing pixels, colour within 1e-4
    on the pixels the oracle classifies well conditioned, and the shares."""
    import numpy as np
    base = oracle.render(wl.scene, wl.camera, wl.W, wl.H, wl.depth, threads=threads)
    ok = oracle.condition(wl.scene, wl.camera, wl.W, wl.H, wl.depth, base=base, threads=threads)
    nongrazing = base.margin >= oracle.GRAZING
    err = np.abs(gpu_rgb - base.rgb).max(1)
    checked = nongrazing & ok
    return {"pixels": int(err.size),
            "id_mismatch_nongrazing": int(((gpu_ids != base.prim_id) & nongrazing).sum()),
            "id_mismatch_all": int((gpu_ids != base.prim_id).sum()),
            "grazing_share": float((~nongrazing).mean()),
            "ill_conditioned_share": float((~ok).mean()),
            "colour_mismatch_frac_nongrazing": float(((err > 1e-4) & nongrazing).sum()
                                                     / max(int(nongrazing.sum()), 1)),
            "colour_mismatch_checked": int(((err > 1e-4) & checked).sum()),
            "max_err_checked": float(err[checked].max()) if checked.any() else 0.0,
            "tolerance": 1e-4}


def cpu_baseline(wl, seconds: float, gpu_rgb=None, gpu_ids=None):
    """The FP64 oracle, as it stands, on this host's cores: whole frames of
    the same workload until `seconds` have passed (at least one).  With the
    GPU's image of that frame, also its parity statistics against the oracle
    (returned separately; not part of the timed sample)."""
    import oracle
    oracle.build()
    threads = oracle.default_threads()
    frames, t0 = 0, time.perf_counter()
    while True:
        oracle.render(wl.scene, wl.camera, wl.W, wl.H, wl.depth, records=False, margins=False,
                      threads=threads)
        frames += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    per_frame = el / frames
    base = {"value": round(wl.W * wl.H / per_frame / 1e6, 4), "unit": "Mrays/s (primary)",
            "cores": threads, "kind": "oracle",
            "sample": f"{frames} whole {wl.W}x{wl.H} frame(s) of the same scene, "
                      f"{per_frame:.3f} s per frame, FP64 C oracle with OpenMP"}
    parity = None
    if gpu_rgb is not None:
        parity = frame_parity(oracle, wl, gpu_rgb, gpu_ids, threads)
    return base, parity


def time_gpu(fn, steps, warmup, stream):
    """Mean GPU time per call of fn() (HIP events on `stream`), in ms."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_steps(step, steps, warmup, stream):
    """The timed region: exactly `steps` calls of step(), after `warmup`,
    bracketed by a synchronize and one HIP event on `stream` on each side,
    with nothing issued between the calls.  Returns (GPU ms per step, host
    wall ms per step)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return e0.elapsed_time(e1) / steps, wall / steps


def time_frames(step, steps, warmup, stream):
    """Per-frame GPU times: one HIP event between consecutive calls of step()
    (steps + 1 events in all), for the distribution of frame times."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    es = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    es[0].record(stream)
    for k in range(steps):
        step()
        es[k + 1].record(stream)
    torch.cuda.synchronize()
    return [es[k].elapsed_time(es[k + 1]) for k in range(steps)]


def time_split(prep, kern, steps, warmup, stream):
    """Per-launch HIP-event times of kern() alone, issued after prep() on
    `stream`: events right before and after each kern() launch, over `steps`
    calls after `warmup`.  Returns the kernel ms list."""
    import torch
    for _ in range(warmup):
        prep()
        kern()
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    ks = [ev() for _ in range(steps)]
    ke = [ev() for _ in range(steps)]
    for k in range(steps):
        prep()
        ks[k].record(stream)
        kern()
        ke[k].record(stream)
    torch.cuda.synchronize()
    return [ks[k].elapsed_time(ke[k]) for k in range(steps)]


def first_render_ms(rt, wl, rgb, stream, uploads=3):
    """The first rt_render of freshly uploaded copies of the scene (no
    recorded tile durations yet: row order), HIP events around the one call;
    the median over `uploads` uploads."""
    import statistics
    import torch
    out = []
    for _ in range(uploads):
        with rt.SceneHandle(wl.scene) as h:
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rt.rt_render(h.handle, wl.camera, wl.W, wl.H, wl.depth, rgb, None, None, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
    return round(statistics.median(out), 5)


def dist(ms):
    """Mean, median, the paper's mean of 10 consecutive frames (the first ten
    timed), min and max of per-frame times (ms)."""
    import statistics
    return {"mean": round(statistics.fmean(ms), 5), "median": round(statistics.median(ms), 5),
            "mean_of_10": round(statistics.fmean(ms[:10]), 5),
            "min": round(min(ms), 5), "max": round(max(ms), 5)}


def work_rates(counts, ms):
    """Tests per second and the fraction of the FP32 peak from the exact tests
    the kernel executed (and the method's algorithmic count per second)."""
    ex = test_flops(counts, True)
    return {"tests_per_s": float("%.4g" % ((counts["sphere_tests"] + counts["plane_tests"])
                                           / (ms * 1e-3))),
            "executed_tests_per_s": float("%.4g" % ((counts["exec_sphere_tests"]
                                                     + counts["exec_plane_tests"]) / (ms * 1e-3))),
            "executed_tflops": round(ex / (ms * 1e-3) / 1e12, 3),
            "executed_frac": round(frac_of_peak(ex, ms), 4)}


def bench_fwd_bwd(rt, scenegen, stream, steps):
    """Differentiable workload (1280x720, 128 spheres, 1 light, depth 3):
    forward render with records + adjoint, and with re-traced decisions."""
    import torch
    prob = scenegen.make_diff_problem()
    wl = prob.workload
    W, H, D = wl.W, wl.H, wl.depth
    h = rt.SceneHandle(wl.scene)
    rgb = torch.empty((H, W, 3), device="cuda")
    grad = torch.ones((H, W, 3), device="cuda")
    N, L = wl.scene.n_spheres, wl.scene.n_lights
    g = {k: torch.empty(sh, device="cuda") for k, sh in (
        ("albedo", (N, 3)), ("refl", (N,)), ("center", (N, 3)), ("light_pos", (L, 3)),
        ("light_int", (L,)))}
    rec = rt.Records(W, H, D)
    counts = rt.render_counts(h.handle, wl.camera, W, H, D)
    t_fwd = time_gpu(lambda: rt.rt_render(h.handle, wl.camera, W, H, D, rgb, None, rec, stream),
                     steps, 5, stream)
    t_bwd = time_gpu(lambda: rt.rt_render_backward(h.handle, wl.camera, W, H, D, grad, g, rec,
                                                   stream), steps, 5, stream)
    t_bwd_re = time_gpu(lambda: rt.rt_render_backward(h.handle, wl.camera, W, H, D, grad, g,
                                                      None, stream), steps, 5, stream)
    t_fwd_plain = time_gpu(lambda: rt.rt_render(h.handle, wl.camera, W, H, D, rgb, None, None,
                                                stream), steps, 5, stream)
    h.close()
    P = W * H
    segs = counts["primary_rays"] + counts["reflection_rays"]
    adj = measured_profile(ADJOINT_FILE, ADJOINT_SOURCES, wl.name)
    bwd_fp32 = None
    if adj.get("executed_fp32_flops_per_launch"):
        f = adj["executed_fp32_flops_per_launch"]
        bwd_fp32 = {"executed_tflops": round(f / (t_bwd * 1e-3) / 1e12, 3),
                    "executed_frac": round(frac_of_peak(f, t_bwd), 4),
                    "source": "FP32 VALU instruction counts x lane utilisation of the adjoint "
                              "kernel, from rocprofv3 (profiles/adjoint_fp32.json)"}
    return {"workload": wl.name,
            "fwd_ms": round(t_fwd, 4), "bwd_ms": round(t_bwd, 4),
            "fwd_bwd_mrays_per_s_checkpoint": round(P / ((t_fwd + t_bwd) * 1e-3) / 1e6, 2),
            "bwd_recompute_ms": round(t_bwd_re, 4),
            "fwd_bwd_mrays_per_s_recompute": round(P / ((t_fwd_plain + t_bwd_re) * 1e-3) / 1e6,
                                                   2),
            "fwd_only_mrays_per_s": round(P / (t_fwd_plain * 1e-3) / 1e6, 2),
            "fwd_work": work_rates(counts, t_fwd_plain),
            "bwd_segments_per_s": float("%.4g" % (segs / (t_bwd * 1e-3))),
            "bwd_fp32": bwd_fp32,
            "work_per_frame": counts}


def adjoint_launches(rt, scenegen, n):
    """The forward+backward workload for a profiler: one render with records,
    then n rt_render_backward launches from them and n re-traced."""
    import torch
    prob = scenegen.make_diff_problem()
    wl = prob.workload
    W, H, D = wl.W, wl.H, wl.depth
    N, L = wl.scene.n_spheres, wl.scene.n_lights
    with rt.SceneHandle(wl.scene) as h:
        rgb = torch.empty((H, W, 3), device="cuda")
        grad = torch.ones((H, W, 3), device="cuda")
        g = {k: torch.empty(sh, device="cuda") for k, sh in (
            ("albedo", (N, 3)), ("refl", (N,)), ("center", (N, 3)), ("light_pos", (L, 3)),
            ("light_int", (L,)))}
        rec = rt.Records(W, H, D)
        rt.rt_render(h.handle, wl.camera, W, H, D, rgb, None, rec)
        for _ in range(n):
            rt.rt_render_backward(h.handle, wl.camera, W, H, D, grad, g, rec)
        for _ in range(n):
            rt.rt_render_backward(h.handle, wl.camera, W, H, D, grad, g, None)
        torch.cuda.synchronize()
    print(json.dumps({"workload": wl.name, "adjoint_launches": n}), flush=True)


def bench_batch(rt, scenegen, stream, steps):
    """64 scenes of uneven size in one graph-captured persistent launch, against
    64 rt_render calls back to back on one stream."""
    import torch
    wls = scenegen.make_batch()
    handles = [rt.SceneHandle(w.scene) for w in wls]
    outs = [torch.empty((w.H, w.W, 3), device="cuda") for w in wls]
    t0 = time.perf_counter()
    b = rt.rt_batch_create([h.handle for h in handles], [w.camera for w in wls],
                           [w.W for w in wls], [w.H for w in wls], [w.depth for w in wls], outs,
                           autotune=True, stream=stream)
    create_s = time.perf_counter() - t0
    counts = rt.batch_counts(b)
    t_graph = time_gpu(lambda: rt.rt_batch_launch(b, stream), steps, 3, stream)

    def sequential():
        for w, h, o in zip(wls, handles, outs):
            rt.rt_render(h.handle, w.camera, w.W, w.H, w.depth, o, None, None, stream)
    t_seq = time_gpu(sequential, steps, 3, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        sequential()
    torch.cuda.synchronize()
    t_seq_wall = (time.perf_counter() - t1) * 1e3 / steps
    shape = rt.rt_batch_shape(b)
    rt.rt_batch_destroy(b)
    for h in handles:
        h.close()
    P = sum(w.W * w.H for w in wls)
    rays = counts["primary_rays"] + counts["reflection_rays"] + counts["shadow_rays"]
    return {"workload": "batch_64scenes", "scenes": len(wls), "pixels": P,
            "graph_ms": round(t_graph, 4), "sequential_ms_gpu": round(t_seq, 4),
            "sequential_ms_wall": round(t_seq_wall, 4),
            "batched_mrays_per_s": round(P / (t_graph * 1e-3) / 1e6, 2),
            "batched_total_mrays_per_s": round(rays / (t_graph * 1e-3) / 1e6, 2),
            "sequential_mrays_per_s": round(P / (max(t_seq, t_seq_wall) * 1e-3) / 1e6, 2),
            "speedup": round(max(t_seq, t_seq_wall) / t_graph, 3),
            "shape": {"workgroups": shape[0], "tile_w": shape[1], "tile_h": shape[2]},
            "create_s": round(create_s, 3),
            "work": work_rates(counts, t_graph), "work_per_launch": counts}


def bench_configs(rt, scenegen, stream, indices=(0, 2), reps=20):
    """The other single-image workloads (the small 256x144 scene and 4K with 512
    spheres): frame time, frames/s, primary Mrays/s, tests per second and the
    fraction of the FP32 peak from the exact tests the kernel executes."""
    out = {}
    for i in indices:
        wl = scenegen.make_workload(i)
        W, H, D = wl.W, wl.H, wl.depth
        h = rt.SceneHandle(wl.scene)
        rgb = torch_empty_image(H, W)
        counts = rt.render_counts(h.handle, wl.camera, W, H, D)
        ms = time_gpu(lambda: rt.rt_render(h.handle, wl.camera, W, H, D, rgb, None, None, stream),
                      reps, 3, stream)
        out[wl.name] = {"ms": round(ms, 4), "fps": round(1e3 / ms, 1),
                        "primary_mrays_per_s": round(W * H / (ms * 1e-3) / 1e6, 1),
                        **work_rates(counts, ms)}
        h.close()
    return out


PAPER_SIZES = ((1280, 720), (1920, 1080), (3840, 2160))


def bench_paper_scene(rt, scenegen, stream, reps=10):
    """The paper's benchmark scene (a seeded stand-in with its shape: one light,
    one plane, five spheres) at 720p, 1080p and 4K in its two settings: one
    shadow sample with one bounce (its GUI runs), and 200 samples of a
    spherical light with three bounces (its non-GUI runs); each with the plain
    background and with a skybox (a procedural 512x256 equirectangular map
    standing in for the paper's HDR image)."""
    s = scenegen.paper_scene()
    h = rt.SceneHandle(s)
    cam = scenegen.Camera()
    out = {"light_radius": scenegen.PAPER_LIGHT_RADIUS, "skybox": "procedural 512x256"}
    for sky in (False, True):
        if sky:
            rt.rt_scene_set_sky(h.handle, scenegen.sky_map())
        for name, (n, D) in scenegen.PAPER_SETTINGS.items():
            res = {}
            for W, H in PAPER_SIZES:
                rgb = torch_empty_image(H, W)
                ms = time_gpu(lambda: rt.rt_render_soft(h.handle, cam, W, H, D, n,
                                                        scenegen.PAPER_LIGHT_RADIUS, rgb, None,
                                                        0, stream), reps, 2, stream)
                res[f"{W}x{H}"] = {"ms": round(ms, 4), "fps": round(1e3 / ms, 1),
                                   "primary_mrays_per_s": round(W * H / (ms * 1e-3) / 1e6, 1)}
            out[name + ("_skybox" if sky else "")] = {"samples": n, "depth": D, **res}
    h.close()
    return out


def bench_interactive(rt, scenegen, stream, frames=60):
    """The paper's interactive loop (its GUI runs, minus the GUI): every frame
    streams new sphere centres (a Verlet step of the five bodies) and a moving
    camera in, renders the paper-scene stand-in with its skybox, and streams
    the image out to pinned host memory (rt_frame_*); frame k+1 is submitted
    before frame k is taken.  Host wall clock per frame, both settings, 720p,
    1080p and 4K, with the paper's 32-bit pixels (packed on the device) and
    with the float image; the median of three runs of `frames` frames."""
    import time
    s = scenegen.paper_scene()
    warm = 4
    motion = scenegen.verlet_motion(s, frames + warm)
    h = rt.SceneHandle(s)
    rt.rt_scene_set_sky(h.handle, scenegen.sky_map())
    out = {"frames": frames, "skybox": "procedural 512x256",
           "motion": "Verlet step of 5 spheres per frame, 1/60 s"}
    R = scenegen.PAPER_LIGHT_RADIUS
    for name, (n, D) in scenegen.PAPER_SETTINGS.items():
        soft = n > 1
        res = {}
        for fmt, fmt_name, bpp in ((rt.RT_FRAME_ARGB8, "argb8", 4),
                                   (rt.RT_FRAME_RGB32F, "rgb32f", 12)):
            for W, H in PAPER_SIZES:
                img = torch_empty_image(H, W)
                f = rt.rt_frame_create(h.handle, W, H, img, soft=soft, stream_out=True, fmt=fmt)

                def run(k0, count):
                    def cam(k):
                        return scenegen.Camera(yaw_deg=-10.0 + 0.3 * k, pitch_deg=-3.0)
                    rad = R if soft else 0.0
                    rt.rt_frame_submit(f, cam(k0), D, n, rad, motion[k0], stream)
                    for k in range(k0 + 1, k0 + count):
                        rt.rt_frame_submit(f, cam(k), D, n, rad, motion[k], stream)
                        rt.rt_frame_result(f)
                    rt.rt_frame_result(f)

                run(0, warm)
                reps = []
                for _ in range(3):   # host-side copies vary between runs: median of three
                    t0 = time.perf_counter()
                    run(warm, frames)
                    reps.append((time.perf_counter() - t0) * 1e3 / frames)
                rt.rt_frame_destroy(f)
                ms = sorted(reps)[1]
                res[f"{fmt_name}_{W}x{H}"] = {"ms": round(ms, 4), "fps": round(1e3 / ms, 1),
                                             "ms_runs": [round(r, 4) for r in reps],
                                             "stream_out_MB": round(W * H * bpp / 1e6, 2)}
        out[name] = {"samples": n, "depth": D, **res}
    h.close()
    return out


def torch_empty_image(H, W):
    import torch
    return torch.empty((H, W, 3), dtype=torch.float32, device="cuda")


# The paper's own frame rates for its render method (one light, one plane, five
# spheres and a skybox, one bounce, GUI-inclusive timing, on the NVIDIA GeForce
# RTX 2060 through TornadoVM/OpenCL).  Context only: another machine, another
# scene and another timing.
PAPER_CONTEXT = {"fps_1280x720": 234, "fps_1920x1080": 152, "fps_3840x2160": 45,
                 "hardware": "NVIDIA GeForce RTX 2060 (TornadoVM, OpenCL backend)",
                 "scene": "1 light, 1 plane, 5 spheres, skybox, 1 bounce, GUI-inclusive",
                 "use": "context only"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", type=int, default=1, choices=[0, 1, 2, 4])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to calibrate HBM byte counters)")
    ap.add_argument("--adjoint-launches", type=int, default=0,
                    help="only run the forward+backward workload: one render with records, "
                         "then this many backward launches from the records and as many "
                         "re-traced (a short run to profile the adjoint kernel), and exit")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline render (no row-order, moving-camera, "
                         "first-render, brute-force, batched or forward+backward "
                         "measurements), so that a profile of the run sees the ordered "
                         "render kernel almost only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the render shards by pixel tiles across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(1)

    import torch
    import paper_2305_07450_amd as rt
    import scenegen

    if args.copy_mib:
        a = torch.ones(args.copy_mib << 18, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.adjoint_launches:
        adjoint_launches(rt, scenegen, args.adjoint_launches)
        return
    wl = scenegen.make_workload(args.workload)
    W, H, D = wl.W, wl.H, wl.depth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = rt.SceneHandle(wl.scene)
    rgb = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    counts = rt.render_counts(h.handle, wl.camera, W, H, D)
    counts_bf = rt.render_counts(h.handle, wl.camera, W, H, D, flags=rt.RT_RENDER_NO_PREFILTER)
    stream = torch.cuda.current_stream()
    ready = rt.RT_RENDER_CONES_READY
    # one step = one rt_render: the eye-cone launch, then the render kernel
    step = lambda: rt.rt_render(h.handle, wl.camera, W, H, D, rgb, None, None, stream)
    torch.cuda.synchronize()
    ms_step_gpu, ms_step_wall = time_steps(step, args.steps, args.warmup, stream)
    ms_step = max(ms_step_wall, ms_step_gpu)
    # outside the timed region: per-frame times (one event between frames),
    # and the render kernel alone, its two launches issued apart so that it
    # gets events of its own
    step_ms = time_frames(step, args.steps, 10, stream)
    prep = lambda: rt.rt_render_prepare(h.handle, wl.camera, W, H, stream)
    kern = lambda: rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, None, None, ready, stream)
    kernel_ms = time_split(prep, kern, args.steps, 10, stream)
    ms_kernel = sum(kernel_ms) / args.steps
    assert torch.isfinite(rgb).all()
    # the tile schedule (tiles longest first, by the durations the previous
    # render of the scene at this size measured): the same loop in row order,
    # the first render of a freshly uploaded scene (row order, recording), and
    # a camera that turns 0.05 degrees a frame (each order measured on the
    # previous, different view)
    schedule = {
        "order": "tiles longest first, by the durations the previous render of the scene at "
                 "this size measured; the first render of a size takes row order"}
    if not args.no_extras:
        row = lambda: rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, None, None,
                                      rt.RT_RENDER_ROW_ORDER, stream)
        row_gpu, row_wall = time_steps(row, args.steps, 10, stream)
        yaws = [0.05 * i for i in range(50)] + [0.05 * (50 - i) for i in range(50)]
        cams = [scenegen.Camera(yaw_deg=y) for y in yaws]
        turn = [0]

        def moving():
            turn[0] += 1
            rt.rt_render(h.handle, cams[turn[0] % len(cams)], W, H, D, rgb, None, None, stream)
        mov_gpu, mov_wall = time_steps(moving, args.steps, 10, stream)
        schedule.update({
            "row_order_ms_per_step": round(max(row_gpu, row_wall), 5),
            "first_render_ms": first_render_ms(rt, wl, rgb, stream),
            "moving_camera_ms_per_step": round(max(mov_gpu, mov_wall), 5),
            "moving_camera": "yaw 0 to 2.45 degrees and back in steps of 0.05 degrees, one "
                             "a frame"})
    ids = torch.empty((H, W), dtype=torch.int32, device=dev)
    rt.rt_render(h.handle, wl.camera, W, H, D, rgb, ids, None, stream)
    torch.cuda.synchronize()
    frame_rgb = rgb.cpu().numpy().reshape(-1, 3).astype("float64")
    frame_ids = ids.cpu().numpy().reshape(-1)

    rays = counts["primary_rays"] + counts["reflection_rays"] + counts["shadow_rays"]
    flops = test_flops(counts, True)
    achieved = flops / (ms_kernel * 1e-3) / 1e12
    prof = measured_profile(TRAFFIC_FILE, KERNEL_SOURCES, wl.name)
    out = {
        "metric": "primary Mrays/s at 1080p (also fps, total Mrays/s, FP32 roofline fraction)",
        "value": round(W * H / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "W": W, "H": H, "spheres": wl.scene.n_spheres,
                   "planes": wl.scene.n_planes, "lights": wl.scene.n_lights, "depth": D,
                   "seed": scenegen.canonical_seed(args.workload), "parallelism": "single-gpu"},
        "fps": round(1e3 / ms_step, 2),
        "total_mrays_per_s": round(rays / (ms_step * 1e-3) / 1e6, 2),
        "step_ms": {"gpu_events": round(ms_step_gpu, 5), "host_wall": round(ms_step_wall, 5)},
        "tile_schedule": schedule,
        "frame_ms": dist(step_ms),
        "render_kernel_ms": dist(kernel_ms),
        **{k: v for k, v in work_rates(counts, ms_step).items()
           if k in ("tests_per_s", "executed_tests_per_s")},
        "work_per_frame": counts,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": prof.get("bytes_per_launch"),
                     "kernel": "render_kernel (culled: cone tests and wave bounds)",
                     "kernel_ms": round(ms_kernel, 5),
                     "flops_per_launch": flops,
                     "executed_fp32": executed_fp32(prof, ms_kernel),
                     "counted": "exact ray-sphere tests x 16 FLOP + ray-plane tests x 12 FLOP "
                                "that the kernel executes, once per ray whose result can still "
                                "matter (rt_render_counts [5], [6])"},
    }
    if not args.no_extras:
        # the method's brute force: the same image without the culling, whose
        # executed tests are exactly the method's algorithmic count
        flags = rt.RT_RENDER_NO_PREFILTER | ready
        bf_kernel = time_split(
            prep, lambda: rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, None, None, flags,
                                          stream), 20, 3, stream)
        ms_bf = sum(bf_kernel) / len(bf_kernel)
        bf_step, _ = time_steps(
            lambda: rt.rt_render_ex(h.handle, wl.camera, W, H, D, rgb, None, None,
                                    rt.RT_RENDER_NO_PREFILTER, stream), 20, 3, stream)
        bf_flops = test_flops(counts_bf, True)
        out["brute_force"] = {
            "kernel": "render_kernel without cone tests and wave bounds (RT_RENDER_NO_PREFILTER)",
            "kernel_ms": round(ms_bf, 5), "step_ms": round(bf_step, 5),
            "flops_per_launch": bf_flops,
            "achieved": round(bf_flops / (ms_bf * 1e-3) / 1e12, 3),
            "frac": round(frac_of_peak(bf_flops, ms_bf), 4),
            "executed_equals_algorithmic": (counts_bf["exec_sphere_tests"]
                                            == counts_bf["sphere_tests"]
                                            and counts_bf["exec_plane_tests"]
                                            == counts_bf["plane_tests"])}
    h.close()
    if not args.no_extras:
        out["fwd_bwd"] = bench_fwd_bwd(rt, scenegen, stream, 20)
        out["batch"] = bench_batch(rt, scenegen, stream, 10)
        out["other_workloads"] = bench_configs(rt, scenegen, stream)
        out["paper_scene"] = bench_paper_scene(rt, scenegen, stream)
        out["interactive"] = bench_interactive(rt, scenegen, stream)
        out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(wl, args.cpu_seconds, frame_rgb,
                                                          frame_ids)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
