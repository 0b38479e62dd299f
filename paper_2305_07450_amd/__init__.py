"""Python binding of librtmi, the MI355X Whitted ray-tracing library.

Argument marshalling only: every step of rendering and differentiation runs
in the HIP kernels behind the C ABI declared in include/rt.h.  The functions
below carry the same names as the C entry points; torch is used for device
memory and streams.  If librtmi.so is not built the import fails: there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtmi.so")

RT_OK, RT_ERR_INVALID_ARG, RT_ERR_OUT_OF_MEMORY, RT_ERR_DEVICE, RT_ERR_UNSUPPORTED = range(5)
RT_HOST, RT_DEVICE = 0, 1
RT_SPEC_BLINN, RT_SPEC_PHONG = 0, 1
RT_MAX_DEPTH = 8
RT_MAX_LIGHTS = 8
RT_MAX_SPHERES = 4096
RT_MAX_PLANES = 16
RT_RENDER_NO_PREFILTER = 1
RT_RENDER_CONES_READY = 2
RT_RENDER_ROW_ORDER = 4
RT_MAX_SAMPLES = 4096
RT_MAX_SKY_DIM = 16384
RT_MAX_DIM = 16384
RT_MAX_BATCH = 4096
RT_FRAME_RGB32F, RT_FRAME_ARGB8 = 0, 1
RT_NUM_COUNTS = 7
RT_STATIC_SCRATCH_BYTES = 16777216

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built: run `python paper_2305_07450_amd/build.py` "
        "(or __graft_entry__.build()); there is no fallback path")


class RtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class rt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("yaw_deg", C.c_float), ("pitch_deg", C.c_float),
                ("fov_deg", C.c_float)]


class rt_scene_desc(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("n_planes", C.c_int32), ("n_lights", C.c_int32),
                ("spec_model", C.c_int32),
                ("sphere_geom", C.c_void_p), ("sphere_mat", C.c_void_p),
                ("sphere_shine", C.c_void_p), ("plane_geom", C.c_void_p),
                ("plane_mat", C.c_void_p), ("plane_shine", C.c_void_p), ("light", C.c_void_p),
                ("ambient", C.c_float), ("spec_strength", C.c_float), ("t_min", C.c_float),
                ("background", C.c_float * 3), ("mem", C.c_int32)]


class rt_records(C.Structure):
    _fields_ = [("ids", C.c_void_p), ("lit", C.c_void_p), ("bytes", C.c_int64)]


class rt_grads(C.Structure):
    _fields_ = [("d_albedo", C.c_void_p), ("d_refl", C.c_void_p), ("d_center", C.c_void_p),
                ("d_light_pos", C.c_void_p), ("d_light_int", C.c_void_p)]


class rt_frame_desc(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("soft", C.c_int32),
                ("stream_out", C.c_int32), ("format", C.c_int32), ("flags", C.c_uint32),
                ("rgb_out", C.c_void_p)]


class rt_frame_input(C.Structure):
    _fields_ = [("cam", rt_camera), ("depth", C.c_int32), ("samples", C.c_int32),
                ("light_radius", C.c_float), ("sphere_pos", C.c_void_p)]


_lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_i32 = C.c_int32
_sig = {
    "rt_scene_upload": (C.c_int, [C.POINTER(rt_scene_desc), _vp, C.POINTER(_vp)]),
    "rt_scene_update": (C.c_int, [_vp, C.POINTER(rt_scene_desc), _vp]),
    "rt_scene_set_sky": (C.c_int, [_vp, _vp, _i32, _i32, C.c_int, _vp]),
    "rt_scene_destroy": (C.c_int, [_vp]),
    "rt_scene_counts": (C.c_int, [_vp, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "rt_records_bytes": (C.c_int64, [_i32, _i32, _i32]),
    "rt_render": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _vp, _vp,
                            C.POINTER(rt_records), _vp]),
    "rt_render_ex": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _vp, _vp,
                               C.POINTER(rt_records), C.c_uint32, _vp]),
    "rt_render_prepare": (C.c_int, [_vp, C.POINTER(rt_camera), C.c_int32, C.c_int32, _vp]),
    "rt_render_soft": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _i32, C.c_float,
                                 _vp, _vp, C.c_uint32, _vp]),
    "rt_render_counts": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _vp, C.c_uint32,
                                   _vp]),
    "rt_render_backward": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _vp,
                                     C.POINTER(rt_records), C.POINTER(rt_grads), _vp]),
    "rt_render_backward_static": (C.c_int, [_vp, C.POINTER(rt_camera), _i32, _i32, _i32, _vp,
                                            C.POINTER(rt_records), C.POINTER(rt_grads), _vp]),
    "rt_batch_create": (C.c_int, [_i32, C.POINTER(_vp), C.POINTER(rt_camera), C.POINTER(_i32),
                                  C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_vp), _i32, _vp,
                                  C.POINTER(_vp)]),
    "rt_batch_launch": (C.c_int, [_vp, _vp]),
    "rt_batch_launch_direct": (C.c_int, [_vp, _vp]),
    "rt_batch_shape": (C.c_int, [_vp, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "rt_batch_counts": (C.c_int, [_vp, _vp, _vp]),
    "rt_batch_destroy": (C.c_int, [_vp]),
    "rt_batch_tune_key": (C.c_int, [_vp, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)]),
    "rt_tune_cache_get": (C.c_int, [C.c_char_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32),
                                    C.POINTER(_i32)]),
    "rt_tune_cache_put": (C.c_int, [C.c_char_p, _i32, _i32, _i32]),
    "rt_tune_cache_forget": (C.c_int, []),
    "rt_frame_create": (C.c_int, [_vp, C.POINTER(rt_frame_desc), C.POINTER(_vp)]),
    "rt_frame_submit": (C.c_int, [_vp, C.POINTER(rt_frame_input), _vp]),
    "rt_frame_result": (C.c_int, [_vp, C.POINTER(_vp)]),
    "rt_frame_destroy": (C.c_int, [_vp]),
    "rt_status_string": (C.c_char_p, [C.c_int]),
    "rt_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _status_name(st: int) -> str:
    return _lib.rt_status_string(st).decode()


def rt_status_string(st: int) -> str:
    return _status_name(st)


def rt_last_error() -> str:
    return _lib.rt_last_error().decode()


def _check(st: int):
    if st != RT_OK:
        raise RtError(st, rt_last_error())


def _stream(stream) -> Optional[int]:
    if stream is None:
        # the null stream when no GPU is visible (argument checks still run)
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr() if t.numel() else None
    return t.ctypes.data if t.size else None


def _dev(t, name: str, dtype: torch.dtype, numel: int, optional: bool = False) -> Optional[int]:
    """Device pointer of a caller-owned buffer, after checking on the host that
    it is a contiguous CUDA tensor of `dtype` holding at least `numel`
    elements: the C side cannot see buffer sizes, so an undersized or
    mistyped buffer would become an out-of-bounds device access.  Raises
    ValueError before any call into the library."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, not {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (CUDA) tensor, not on {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < max(int(numel), 0):
        raise ValueError(f"{name} holds {t.numel()} elements, {int(numel)} needed")
    return t.data_ptr() if t.numel() else None


def _records_arg(rec, W: int, H: int, depth: int):
    """rt_records of a Records object after checking it covers W x H x (depth+1)."""
    if rec is None:
        return None
    if not isinstance(rec, Records):
        raise ValueError("rec must be a Records object")
    _dev(rec.buf, "records", torch.uint8, 0)
    need = (int(depth) + 1) * int(W) * int(H)
    if rec.n < need:
        raise ValueError(f"records hold {rec.n} pixel-segments, {need} needed")
    return C.byref(rec.c)


def rt_scene_counts(handle: int):
    """(n_spheres, n_planes, n_lights) of an uploaded scene."""
    n, p, l = _i32(), _i32(), _i32()
    _check(_lib.rt_scene_counts(handle, C.byref(n), C.byref(p), C.byref(l)))
    return n.value, p.value, l.value


def make_camera(cam) -> rt_camera:
    """rt_camera from any object with eye, yaw_deg, pitch_deg, fov_deg."""
    return rt_camera((C.c_float * 3)(*[float(v) for v in cam.eye]), float(cam.yaw_deg),
                     float(cam.pitch_deg), float(cam.fov_deg))


class _Desc:
    """rt_scene_desc plus the arrays it points to (kept alive for the call)."""

    def __init__(self, scene, arrays: Optional[Dict[str, object]] = None):
        get = (lambda k: arrays[k]) if arrays is not None else (lambda k: getattr(scene, k))
        names = ("sphere_geom", "sphere_mat", "sphere_shine", "plane_geom", "plane_mat",
                 "plane_shine", "light")
        vals = [get(k) for k in names]
        on_dev = [isinstance(v, torch.Tensor) and v.is_cuda for v in vals]
        if any(on_dev) and not all(on_dev):
            raise ValueError("scene arrays must be all host or all device arrays")
        if all(on_dev):
            vals = [v.detach().to(torch.float32).contiguous() for v in vals]
            mem = RT_DEVICE
        else:
            vals = [np.ascontiguousarray(np.asarray(v, dtype=np.float32)) for v in vals]
            mem = RT_HOST
        self.keep = vals
        n_sph = int(vals[0].shape[0]) if vals[0].ndim else 0
        n_pl = int(vals[3].shape[0]) if vals[3].ndim else 0
        n_l = int(vals[6].shape[0]) if vals[6].ndim else 0
        # the library reads exactly these many floats from each array
        for name, v, want in zip(names, vals, (4 * n_sph, 4 * n_sph, n_sph, 4 * n_pl, 4 * n_pl,
                                                n_pl, 4 * n_l)):
            got = int(v.numel() if isinstance(v, torch.Tensor) else v.size)
            if got != want:
                raise ValueError(f"scene array {name} has {got} values, {want} expected")
        self.c = rt_scene_desc(
            n_sph, n_pl, n_l, int(scene.spec_model),
            *[_ptr(v) for v in vals],
            float(scene.ambient), float(scene.spec_strength), float(scene.t_min),
            (C.c_float * 3)(*[float(v) for v in scene.background]), mem)


def rt_scene_upload(scene, stream=None, arrays: Optional[Dict[str, object]] = None) -> int:
    """Upload a scene (numpy arrays -> RT_HOST, CUDA tensors -> RT_DEVICE);
    returns the opaque rt_scene handle (int)."""
    d = _Desc(scene, arrays)
    h = _vp()
    _check(_lib.rt_scene_upload(C.byref(d.c), _stream(stream), C.byref(h)))
    return h.value


def rt_scene_update(handle: int, scene, stream=None, arrays: Optional[Dict[str, object]] = None):
    d = _Desc(scene, arrays)
    _check(_lib.rt_scene_update(handle, C.byref(d.c), _stream(stream)))
    return d   # caller keeps device arrays alive until the stream has consumed them


def rt_scene_set_sky(handle: int, rgb=None, stream=None):
    """Give the scene a skybox, float32 [h, w, 3] (numpy -> RT_HOST, CUDA
    tensor -> RT_DEVICE), or remove it (rgb None)."""
    if rgb is None:
        _check(_lib.rt_scene_set_sky(handle, None, 0, 0, 0, _stream(stream)))
        return None
    if isinstance(rgb, torch.Tensor):
        if rgb.dtype != torch.float32 or not rgb.is_contiguous() or rgb.dim() != 3 \
                or rgb.shape[2] != 3:
            raise ValueError("skybox tensor must be contiguous float32 [h, w, 3]")
        arr, mem = rgb, 1 if rgb.is_cuda else 0
    else:
        arr = np.ascontiguousarray(rgb, dtype=np.float32)
        if arr.ndim != 3 or arr.shape[2] != 3:
            raise ValueError("skybox must be [h, w, 3]")
        mem = 0
    _check(_lib.rt_scene_set_sky(handle, _ptr(arr), int(arr.shape[1]), int(arr.shape[0]), mem,
                                 _stream(stream)))
    return arr   # with RT_DEVICE the caller keeps it alive until the stream has consumed it


def rt_scene_destroy(handle: int):
    _check(_lib.rt_scene_destroy(handle))


def rt_records_bytes(W: int, H: int, depth: int) -> int:
    return int(_lib.rt_records_bytes(W, H, depth))


class Records:
    """Caller-owned device records: ids int32 [depth+1, H, W], lit uint8 [depth+1, H, W]."""

    def __init__(self, W: int, H: int, depth: int, device="cuda"):
        n = (depth + 1) * H * W
        self.n = n
        self.buf = torch.empty(rt_records_bytes(W, H, depth), dtype=torch.uint8, device=device)
        self.ids = self.buf[:4 * n].view(torch.int32).view(depth + 1, H, W)
        self.lit = self.buf[4 * n:].view(depth + 1, H, W)
        self.c = rt_records(self.ids.data_ptr(), self.lit.data_ptr(), self.buf.numel())


def _image_args(W: int, H: int, rgb_out, id_out):
    P = int(W) * int(H)
    return (_dev(rgb_out, "rgb_out", torch.float32, 3 * P),
            _dev(id_out, "id_out", torch.int32, P, optional=True))


def rt_render(handle: int, camera, W: int, H: int, depth: int, rgb_out: torch.Tensor,
              id_out: Optional[torch.Tensor] = None, rec: Optional[Records] = None,
              stream=None):
    cam = make_camera(camera)
    rgb_p, id_p = _image_args(W, H, rgb_out, id_out)
    rec_p = _records_arg(rec, W, H, depth)
    _check(_lib.rt_render(handle, C.byref(cam), W, H, depth, rgb_p, id_p, rec_p,
                          _stream(stream)))


def rt_render_ex(handle: int, camera, W: int, H: int, depth: int, rgb_out: torch.Tensor,
                 id_out: Optional[torch.Tensor] = None, rec: Optional["Records"] = None,
                 flags: int = 0, stream=None):
    cam = make_camera(camera)
    rgb_p, id_p = _image_args(W, H, rgb_out, id_out)
    rec_p = _records_arg(rec, W, H, depth)
    _check(_lib.rt_render_ex(handle, C.byref(cam), W, H, depth, rgb_p, id_p, rec_p, int(flags),
                             _stream(stream)))


# algorithmic tests, rays, then the tests the kernel executes (include/rt.h)
def rt_render_prepare(handle: int, camera, W: int, H: int, stream=None):
    """The preparation launch of rt_render on its own: eye cones and the tile
    order of a W x H image (see RT_RENDER_CONES_READY)."""
    cam = make_camera(camera)
    _check(_lib.rt_render_prepare(handle, C.byref(cam), int(W), int(H), _stream(stream)))


COUNT_NAMES = ("sphere_tests", "plane_tests", "primary_rays", "reflection_rays", "shadow_rays",
               "exec_sphere_tests", "exec_plane_tests")


def rt_render_soft(handle: int, camera, W: int, H: int, depth: int, samples: int,
                   light_radius: float, rgb_out: torch.Tensor,
                   id_out: Optional[torch.Tensor] = None, flags: int = 0, stream=None):
    """Soft shadows: every light a sphere of radius light_radius sampled at
    `samples` points (see include/rt.h)."""
    cam = make_camera(camera)
    rgb_p, id_p = _image_args(W, H, rgb_out, id_out)
    _check(_lib.rt_render_soft(handle, C.byref(cam), W, H, depth, int(samples),
                               float(light_radius), rgb_p, id_p, int(flags), _stream(stream)))


def rt_render_counts(handle: int, camera, W: int, H: int, depth: int, counts: torch.Tensor,
                     flags: int = 0, stream=None):
    """Add the work counters of one render to counts (int64 [RT_NUM_COUNTS]);
    flags = RT_RENDER_NO_PREFILTER counts the kernel without the culling."""
    cam = make_camera(camera)
    cnt_p = _dev(counts, "counts", torch.int64, RT_NUM_COUNTS)
    _check(_lib.rt_render_counts(handle, C.byref(cam), W, H, depth, cnt_p, int(flags),
                                 _stream(stream)))


def render_counts(handle: int, camera, W: int, H: int, depth: int,
                  flags: int = 0) -> Dict[str, int]:
    c = torch.zeros(RT_NUM_COUNTS, dtype=torch.int64, device="cuda")
    rt_render_counts(handle, camera, W, H, depth, c, flags)
    return dict(zip(COUNT_NAMES, c.cpu().tolist()))


def rt_render_backward(handle: int, camera, W: int, H: int, depth: int, grad_rgb: torch.Tensor,
                       grads: Dict[str, torch.Tensor], rec: Optional[Records] = None,
                       stream=None):
    cam = make_camera(camera)
    grad_p = _dev(grad_rgb, "grad_rgb", torch.float32, 3 * int(W) * int(H))
    rec_p = _records_arg(rec, W, H, depth)
    g = _grads_arg(handle, grads)
    _check(_lib.rt_render_backward(handle, C.byref(cam), W, H, depth, grad_p, rec_p, C.byref(g),
                                   _stream(stream)))


def rt_render_backward_static(handle: int, camera, W: int, H: int, depth: int,
                              grad_rgb: torch.Tensor, grads: Dict[str, torch.Tensor],
                              rec: Optional[Records] = None, stream=None):
    cam = make_camera(camera)
    grad_p = _dev(grad_rgb, "grad_rgb", torch.float32, 3 * int(W) * int(H))
    rec_p = _records_arg(rec, W, H, depth)
    g = _grads_arg(handle, grads)
    _check(_lib.rt_render_backward_static(handle, C.byref(cam), W, H, depth, grad_p, rec_p,
                                          C.byref(g), _stream(stream)))


GRAD_NAMES = ("albedo", "refl", "center", "light_pos", "light_int")


def _grads_arg(handle: int, grads: Dict[str, torch.Tensor]) -> rt_grads:
    """rt_grads from a dict of device float32 tensors (missing or None entries
    are skipped), each checked against the scene's counts."""
    unknown = set(grads) - set(GRAD_NAMES)
    if unknown:
        raise ValueError(f"unknown gradient groups {sorted(unknown)}")
    N, _, L = rt_scene_counts(handle)
    sizes = dict(albedo=3 * N, refl=N, center=3 * N, light_pos=3 * L, light_int=L)
    return rt_grads(*[_dev(grads.get(k), f"grads[{k!r}]", torch.float32, sizes[k],
                           optional=True) for k in GRAD_NAMES])


def rt_batch_create(handles: Sequence[int], cameras, W: Sequence[int], H: Sequence[int],
                    depth: Sequence[int], rgb_outs: Sequence[torch.Tensor], autotune: bool = True,
                    stream=None) -> int:
    n = len(handles)
    if not (len(cameras) == len(W) == len(H) == len(depth) == len(rgb_outs) == n):
        raise ValueError("batch arrays differ in length")
    cams = (rt_camera * n)(*[make_camera(c) for c in cameras])
    arr = lambda v: (_i32 * n)(*[int(x) for x in v])
    outs = (_vp * n)(*[_dev(t, f"rgb_outs[{i}]", torch.float32, 3 * int(w) * int(h))
                       for i, (t, w, h) in enumerate(zip(rgb_outs, W, H))])
    hs = (_vp * n)(*handles)
    b = _vp()
    _check(_lib.rt_batch_create(n, hs, cams, arr(W), arr(H), arr(depth), outs, int(autotune),
                                _stream(stream), C.byref(b)))
    return b.value


def rt_batch_launch(batch: int, stream=None):
    _check(_lib.rt_batch_launch(batch, _stream(stream)))


def rt_batch_launch_direct(batch: int, stream=None):
    _check(_lib.rt_batch_launch_direct(batch, _stream(stream)))


def rt_batch_counts(batch: int, counts: torch.Tensor, stream=None):
    """Add the work counters of one (direct) batch launch to counts (int64
    [RT_NUM_COUNTS])."""
    _check(_lib.rt_batch_counts(batch, _dev(counts, "counts", torch.int64, RT_NUM_COUNTS),
                                _stream(stream)))


def batch_counts(batch: int) -> Dict[str, int]:
    c = torch.zeros(RT_NUM_COUNTS, dtype=torch.int64, device="cuda")
    rt_batch_counts(batch, c)
    return dict(zip(COUNT_NAMES, c.cpu().tolist()))


def rt_batch_shape(batch: int):
    g, tw, th = _i32(), _i32(), _i32()
    _check(_lib.rt_batch_shape(batch, C.byref(g), C.byref(tw), C.byref(th)))
    return g.value, tw.value, th.value


def rt_batch_destroy(batch: int):
    _check(_lib.rt_batch_destroy(batch))


def rt_batch_tune_key(batch: int) -> str:
    n = C.c_int64()
    _check(_lib.rt_batch_tune_key(batch, None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value + 1)
    _check(_lib.rt_batch_tune_key(batch, buf, n.value + 1, C.byref(n)))
    return buf.value.decode()


def rt_tune_cache_get(key: str):
    """(workgroups, tile_w, tile_h) cached for `key`, or None."""
    g, tw, th, found = _i32(), _i32(), _i32(), _i32()
    _check(_lib.rt_tune_cache_get(key.encode(), C.byref(g), C.byref(tw), C.byref(th),
                                  C.byref(found)))
    return (g.value, tw.value, th.value) if found.value else None


def rt_tune_cache_put(key: str, workgroups: int, tile_w: int, tile_h: int):
    _check(_lib.rt_tune_cache_put(key.encode(), workgroups, tile_w, tile_h))


def rt_tune_cache_forget():
    _check(_lib.rt_tune_cache_forget())


def rt_frame_create(handle: int, W: int, H: int, rgb_out: torch.Tensor, soft: bool = False,
                    stream_out: bool = False, fmt: int = 0, flags: int = 0) -> int:
    """Interactive per-frame path for one scene and image size (see
    include/rt.h); rgb_out is the device image every frame renders into, fmt
    the streamed-out format (RT_FRAME_RGB32F or RT_FRAME_ARGB8)."""
    d = rt_frame_desc(int(W), int(H), int(bool(soft)), int(bool(stream_out)), int(fmt),
                      int(flags), _dev(rgb_out, "rgb_out", torch.float32, 3 * int(W) * int(H)))
    f = _vp()
    _check(_lib.rt_frame_create(handle, C.byref(d), C.byref(f)))
    _frame_spheres[f.value] = rt_scene_counts(handle)[0]
    return f.value


# spheres of each frame object's scene, to check the centres of every submit
_frame_spheres: Dict[int, int] = {}


def rt_frame_submit(frame: int, camera, depth: int, samples: int = 1, light_radius: float = 0.0,
                    sphere_pos=None, stream=None):
    """Stage and launch one frame; sphere_pos is a host float32 [N, 3] array of
    new centres, or None to keep them."""
    pos = None
    if sphere_pos is not None:
        pos = np.ascontiguousarray(sphere_pos, dtype=np.float32)
        want = 3 * _frame_spheres.get(frame, pos.size // 3)
        if pos.size != want:
            raise ValueError(f"sphere_pos has {pos.size} values, {want} expected")
    inp = rt_frame_input(make_camera(camera), int(depth), int(samples), float(light_radius),
                         _ptr(pos) if pos is not None else None)
    _check(_lib.rt_frame_submit(frame, C.byref(inp), _stream(stream)))


def rt_frame_result(frame: int, W: int = 0, H: int = 0, fmt: int = 0):
    """Wait for the oldest frame not yet returned.  With stream_out, returns a
    numpy view of its pinned host image (valid until the second submit after
    the frame's own): float32 [H, W, 3] for RT_FRAME_RGB32F, uint32 [H, W]
    for RT_FRAME_ARGB8; otherwise None."""
    p = _vp()
    _check(_lib.rt_frame_result(frame, C.byref(p)))
    if not p.value:
        return None
    if fmt == RT_FRAME_ARGB8:
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint32)), shape=(int(H), int(W)))
    return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_float)), shape=(int(H), int(W), 3))


def rt_frame_destroy(frame: int):
    _frame_spheres.pop(frame, None)
    _check(_lib.rt_frame_destroy(frame))


# ---------------------------------------------------------------- helpers

class SceneHandle:
    """Owns one uploaded scene; frees it on close()/garbage collection."""

    def __init__(self, scene, stream=None):
        self.scene = scene
        self.handle = rt_scene_upload(scene, stream)
        self.n_spheres = int(np.asarray(scene.sphere_geom).reshape(-1, 4).shape[0]) \
            if not isinstance(scene.sphere_geom, torch.Tensor) else int(scene.sphere_geom.shape[0])
        self.n_lights = int(np.asarray(scene.light).reshape(-1, 4).shape[0]) \
            if not isinstance(scene.light, torch.Tensor) else int(scene.light.shape[0])

    def close(self):
        if self.handle:
            rt_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def render(handle: int, camera, W: int, H: int, depth: int, ids: bool = False,
           records: bool = False, stream=None, device="cuda"):
    """Allocate outputs and call rt_render.  Returns (rgb [H,W,3], ids [H,W] or
    None, Records or None)."""
    rgb = torch.empty((H, W, 3), dtype=torch.float32, device=device)
    idt = torch.empty((H, W), dtype=torch.int32, device=device) if ids else None
    rec = Records(W, H, depth, device) if records else None
    rt_render(handle, camera, W, H, depth, rgb, idt, rec, stream)
    return rgb, idt, rec


from .autograd import RTRender, render_differentiable  # noqa: E402,F401
