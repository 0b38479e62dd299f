"""FP64 CPU oracle for the Whitted ray tracer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path (the
HIP library and its binding in ``paper_2305_07450_amd``) never imports it, and it
shares no code with the HIP kernels: the only common module is ``scenegen``,
which draws random numbers and holds no rendering arithmetic.

Contents:
  * ``rt_oracle.c``  - plain C, FP64, OpenMP over pixels: cameras, intersections,
    closest hit, cast shadows, Blinn/Phong shading, recursive reflections, the
    primary decision margin and the algorithmic test/ray counters.
  * this module      - ctypes binding, the conditioning classifier built on
    jittered re-traces, and per-pixel helpers.
  * ``grad_ref.py``  - fixed-visibility re-shade in torch float64 on the CPU,
    differentiated by autograd (the reference gradient).

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, the paper's worked example,
brute force or exact arithmetic, except colour at arbitrary pixels of general
scenes beyond those checks ("parity unpinned" there: the oracle is itself the
reference).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from scenegen import Camera, Scene

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rt_oracle.c")
LIB = os.path.join(HERE, "librt_oracle.so")

MISS = -1
NOT_TRACED = -2
SPEC_BLINN, SPEC_PHONG = 0, 1
CNT_NAMES = ("sphere_tests", "plane_tests", "primary_rays", "reflection_rays", "shadow_rays")

# Conditioning: K re-traces with each segment's ray perturbed by JITTER
# (relative, 4 FP32 ulps); a pixel is ill-conditioned when its colour spread
# exceeds COND_SPREAD or any re-trace takes a different discrete decision.
# An FP32 kernel whose rounding moves each ray by up to ~16 ulps then stays
# within 4 x COND_SPREAD = 1e-4 on the pixels classified well conditioned.
JITTER = 2.0 ** -21
COND_RUNS = 8
COND_SPREAD = 2.5e-5
GRAZING = 1e-6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "rt_oracle.h"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Scene(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("n_planes", C.c_int32), ("n_lights", C.c_int32),
                ("spec_model", C.c_int32),
                ("sphere_geom", C.c_void_p), ("sphere_mat", C.c_void_p),
                ("sphere_shine", C.c_void_p), ("plane_geom", C.c_void_p),
                ("plane_mat", C.c_void_p), ("plane_shine", C.c_void_p), ("light", C.c_void_p),
                ("ambient", C.c_double), ("spec_strength", C.c_double), ("t_min", C.c_double),
                ("background", C.c_double * 3), ("shadow_samples", C.c_int32),
                ("light_radius", C.c_double), ("sky", C.c_void_p), ("sky_w", C.c_int32),
                ("sky_h", C.c_int32)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("yaw_deg", C.c_double), ("pitch_deg", C.c_double),
                ("fov_deg", C.c_double)]


class _Outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("prim_id", C.c_void_p), ("seg_id", C.c_void_p),
                ("lit", C.c_void_p), ("margin", C.c_void_p), ("counts", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.or_render_pixels.restype = C.c_int
        _lib.or_render_pixels.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_int32,
                                          C.c_int32, C.c_int32, C.c_int64, C.c_void_p,
                                          C.c_double, C.c_uint64, C.c_int32,
                                          C.POINTER(_Outputs)]
        _lib.or_camera_rays.restype = None
        _lib.or_camera_rays.argtypes = [C.POINTER(_Camera), C.c_int32, C.c_int32, C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.or_closest_hits.restype = None
        _lib.or_closest_hits.argtypes = [C.POINTER(_Scene), C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        _lib.or_sphere_root.restype = C.c_int
        _lib.or_sphere_root.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                        C.POINTER(C.c_double)]
        _lib.or_plane_root.restype = C.c_int
        _lib.or_plane_root.argtypes = _lib.or_sphere_root.argtypes
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


class Scene64:
    """FP64 copy of a scene, so that finite differences can move a parameter
    by amounts FP32 cannot hold.  Same attribute names as scenegen.Scene."""

    ARRAYS = ("sphere_geom", "sphere_mat", "sphere_shine", "plane_geom", "plane_mat",
              "plane_shine", "light")

    def __init__(self, scene):
        for k in self.ARRAYS:
            setattr(self, k, np.array(getattr(scene, k), dtype=np.float64))
        for k in ("ambient", "spec_strength", "t_min", "spec_model"):
            setattr(self, k, getattr(scene, k))
        self.background = tuple(float(v) for v in scene.background)

    n_spheres = property(lambda self: int(self.sphere_geom.shape[0]))
    n_planes = property(lambda self: int(self.plane_geom.shape[0]))
    n_lights = property(lambda self: int(self.light.shape[0]))

    def copy(self):
        return Scene64(self)


class _Pack:
    """Scene promoted exactly from FP32 to FP64, kept alive for the C call;
    `samples` > 1 and `light_radius` select soft shadows."""

    def __init__(self, s: Scene, samples: int = 1, light_radius: float = 0.0, sky=None):
        self.arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in (
            s.sphere_geom, s.sphere_mat, s.sphere_shine, s.plane_geom, s.plane_mat,
            s.plane_shine, s.light)]
        a = self.arrays
        self.sky = (np.ascontiguousarray(sky, dtype=np.float64) if sky is not None
                    else np.zeros((0, 0, 3)))
        self.c = _Scene(s.n_spheres, s.n_planes, s.n_lights, int(s.spec_model),
                        _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(a[3]), _ptr(a[4]), _ptr(a[5]),
                        _ptr(a[6]), float(s.ambient), float(s.spec_strength), float(s.t_min),
                        (C.c_double * 3)(*[float(v) for v in s.background]), int(samples),
                        float(light_radius), _ptr(self.sky), int(self.sky.shape[1]),
                        int(self.sky.shape[0]))


def _cam(cam: Camera) -> _Camera:
    return _Camera((C.c_double * 3)(*[float(v) for v in cam.eye]), float(cam.yaw_deg),
                   float(cam.pitch_deg), float(cam.fov_deg))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


class Result(dict):
    """Oracle outputs for the requested pixels (dict with attribute access)."""

    __getattr__ = dict.__getitem__


def render(scene: Scene, cam: Camera, W: int, H: int, depth: int,
           pixels: Optional[np.ndarray] = None, records: bool = True, margins: bool = True,
           jitter: float = 0.0, seed: int = 0, threads: Optional[int] = None,
           samples: int = 1, light_radius: float = 0.0, sky=None) -> Result:
    """Render the listed pixels (flat indices y*W+x; default all) in FP64;
    samples > 1 renders soft shadows of lights of radius light_radius; `sky`
    (an [h, w, 3] map) replaces the background colour of misses.

    Returns rgb [n,3] float64, prim_id [n], seg_id [n,depth+1], lit [n,depth+1],
    margin [n] and the algorithmic counters (dict)."""
    pix = (np.arange(W * H, dtype=np.int64) if pixels is None
           else np.ascontiguousarray(pixels, dtype=np.int64).reshape(-1))
    n = pix.size
    rgb = np.zeros((n, 3), np.float64)
    prim = np.zeros(n, np.int32)
    seg = np.zeros((n, depth + 1), np.int32) if records else np.zeros(0, np.int32)
    lit = np.zeros((n, depth + 1), np.uint32) if records else np.zeros(0, np.uint32)
    mar = np.zeros(n, np.float64) if margins else np.zeros(0, np.float64)
    cnt = np.zeros(len(CNT_NAMES), np.int64)
    sp = _Pack(scene, samples, light_radius, sky)
    out = _Outputs(_ptr(rgb), _ptr(prim), _ptr(seg) if records else 0,
                   _ptr(lit) if records else 0, _ptr(mar) if margins else 0, _ptr(cnt))
    rc = lib().or_render_pixels(C.byref(sp.c), C.byref(_cam(cam)), W, H, depth, n, _ptr(pix),
                                float(jitter), int(seed) & (2**64 - 1),
                                int(threads or default_threads()), C.byref(out))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    r = Result(rgb=rgb, prim_id=prim, counts=dict(zip(CNT_NAMES, cnt.tolist())), pixels=pix)
    if records:
        r["seg_id"], r["lit"] = seg, lit
    if margins:
        r["margin"] = mar
    return r


def condition(scene: Scene, cam: Camera, W: int, H: int, depth: int,
              pixels: Optional[np.ndarray] = None, base: Optional[Result] = None,
              runs: int = COND_RUNS, jitter: float = JITTER, spread: float = COND_SPREAD,
              threads: Optional[int] = None, samples: int = 1,
              light_radius: float = 0.0, sky=None) -> np.ndarray:
    """Boolean mask of well-conditioned pixels: every jittered re-trace keeps
    the same decision record and the colour spread stays within `spread`.
    With soft shadows every sample ray moves with its segment, so a pixel
    whose visible sample count changes shows a colour spread."""
    if base is None:
        base = render(scene, cam, W, H, depth, pixels, threads=threads, samples=samples,
                      light_radius=light_radius, sky=sky)
    ok = np.ones(base.rgb.shape[0], bool)
    lo, hi = base.rgb.copy(), base.rgb.copy()
    for k in range(runs):
        r = render(scene, cam, W, H, depth, base.pixels, margins=False, jitter=jitter,
                   seed=0x5EED0000 + k, threads=threads, samples=samples,
                   light_radius=light_radius, sky=sky)
        ok &= (r.seg_id == base.seg_id).all(1) & (r.lit == base.lit).all(1)
        lo = np.minimum(lo, r.rgb)
        hi = np.maximum(hi, r.rgb)
    ok &= (hi - lo).max(1) <= spread
    return ok


def camera_rays(cam: Camera, W: int, H: int, pixels: np.ndarray):
    pix = np.ascontiguousarray(pixels, dtype=np.int64).reshape(-1)
    o = np.zeros((pix.size, 3))
    d = np.zeros((pix.size, 3))
    lib().or_camera_rays(C.byref(_cam(cam)), W, H, pix.size, _ptr(pix), _ptr(o), _ptr(d))
    return o, d


def closest_hits(scene: Scene, o: np.ndarray, d: np.ndarray):
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    ids = np.zeros(o.shape[0], np.int32)
    ts = np.zeros(o.shape[0], np.float64)
    sp = _Pack(scene)
    lib().or_closest_hits(C.byref(sp.c), o.shape[0], _ptr(o), _ptr(d), _ptr(ids), _ptr(ts))
    return ids, ts


def sphere_root(o, d, geom4, t_min):
    o, d, g = (np.ascontiguousarray(v, dtype=np.float64) for v in (o, d, geom4))
    t = C.c_double(0.0)
    hit = lib().or_sphere_root(_ptr(o), _ptr(d), _ptr(g), float(t_min), C.byref(t))
    return (t.value if hit else None)


def plane_root(o, d, geom4, t_min):
    o, d, g = (np.ascontiguousarray(v, dtype=np.float64) for v in (o, d, geom4))
    t = C.c_double(0.0)
    hit = lib().or_plane_root(_ptr(o), _ptr(d), _ptr(g), float(t_min), C.byref(t))
    return (t.value if hit else None)


def id_edges(prim_id: np.ndarray, W: int, H: int, radius: int = 2) -> np.ndarray:
    """Pixels within Chebyshev distance `radius` of a primary-ID change (full frame)."""
    ids = prim_id.reshape(H, W)
    edge = np.zeros((H, W), bool)
    edge[:, 1:] |= ids[:, 1:] != ids[:, :-1]
    edge[:, :-1] |= ids[:, 1:] != ids[:, :-1]
    edge[1:, :] |= ids[1:, :] != ids[:-1, :]
    edge[:-1, :] |= ids[1:, :] != ids[:-1, :]
    out = edge.copy()
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            if dx == 0 and dy == 0:
                continue
            sh = np.zeros_like(edge)
            ys = slice(max(dy, 0), H + min(dy, 0))
            yd = slice(max(-dy, 0), H + min(-dy, 0))
            xs = slice(max(dx, 0), W + min(dx, 0))
            xd = slice(max(-dx, 0), W + min(-dx, 0))
            sh[yd, xd] = edge[ys, xs]
            out |= sh
    return out.reshape(-1)
