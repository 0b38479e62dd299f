"""C ABI checks that need no GPU: the library loads, exports every entry
point that include/rt.h declares, and rejects bad arguments on the host before
any HIP call."""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import scenegen
from scenegen import Camera

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rt():
    import paper_2305_07450_amd as rt
    return rt


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(rt_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("rt_scene_upload", "rt_scene_update", "rt_scene_destroy", "rt_records_bytes",
              "rt_render", "rt_render_counts", "rt_render_backward", "rt_batch_create",
              "rt_batch_launch", "rt_batch_destroy", "rt_status_string", "rt_last_error"):
        assert s in syms


def test_binding_constants_match_the_header(rt):
    """Every numeric #define and enum value of include/rt.h has a constant of
    the same name and value in the Python binding."""
    text = open(os.path.join(ROOT, "include", "rt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    consts = {m[0]: int(m[1]) for m in re.findall(r"^#define\s+(RT_\w+)\s+(\d+)[uU]?\s*$", text,
                                                  flags=re.M)}
    consts.update({m[0]: int(m[1]) for m in re.findall(r"\b(RT_[A-Z0-9_]+)\s*=\s*(\d+)", text)})
    assert len(consts) >= 20, sorted(consts)
    for name, value in consts.items():
        assert getattr(rt, name, None) == value, name


def test_library_exports_every_declared_symbol(rt):
    lib = C.CDLL(rt.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol(rt):
    missing = [s for s in declared_symbols() if not hasattr(rt, s)]
    assert not missing, missing


def test_status_strings(rt):
    assert rt.rt_status_string(0) == "RT_OK"
    assert rt.rt_status_string(1) == "RT_ERR_INVALID_ARG"
    assert rt.rt_status_string(4) == "RT_ERR_UNSUPPORTED"


def test_records_bytes(rt):
    assert rt.rt_records_bytes(1920, 1080, 4) == 1920 * 1080 * 5 * 5
    assert rt.rt_records_bytes(0, 10, 1) == -1
    assert rt.rt_records_bytes(10, 10, 9) == -1
    assert rt.rt_records_bytes(10, 10, -1) == -1


def _bad_scenes():
    base = scenegen.tiny_scene(1, n_spheres=3, n_lights=2)
    out = []

    def mod(name, f):
        s = base.copy()
        f(s)
        out.append((name, s))

    mod("radius_zero", lambda s: s.sphere_geom.__setitem__((0, 3), 0.0))
    mod("radius_negative", lambda s: s.sphere_geom.__setitem__((1, 3), -1.0))
    mod("nan_centre", lambda s: s.sphere_geom.__setitem__((0, 0), np.nan))
    mod("inf_albedo", lambda s: s.sphere_mat.__setitem__((2, 1), np.inf))
    mod("zero_exponent", lambda s: s.sphere_shine.__setitem__(0, 0.0))
    mod("plane_not_unit", lambda s: s.plane_geom.__setitem__((0, 1), 2.0))
    mod("negative_light", lambda s: s.light.__setitem__((1, 3), -0.5))
    mod("nan_light", lambda s: s.light.__setitem__((0, 2), np.nan))
    mod("negative_tmin", lambda s: setattr(s, "t_min", -1.0))
    mod("bad_spec_model", lambda s: setattr(s, "spec_model", 7))
    mod("nan_ambient", lambda s: setattr(s, "ambient", float("nan")))
    return out


@pytest.mark.parametrize("name,scene", _bad_scenes(), ids=[n for n, _ in _bad_scenes()])
def test_upload_rejects_bad_values_before_any_device_call(rt, name, scene):
    with pytest.raises(rt.RtError) as e:
        rt.rt_scene_upload(scene, stream=0)
    assert e.value.status == rt.RT_ERR_INVALID_ARG, str(e.value)


def test_upload_rejects_bad_counts(rt):
    s = scenegen.tiny_scene(1, n_spheres=3, n_lights=1)
    d = rt._Desc(s)
    for field, val in (("n_spheres", -1), ("n_spheres", rt.RT_MAX_SPHERES + 1),
                       ("n_planes", rt.RT_MAX_PLANES + 1), ("n_lights", rt.RT_MAX_LIGHTS + 1),
                       ("mem", 5)):
        c = rt.rt_scene_desc.from_buffer_copy(d.c)
        setattr(c, field, val)
        h = C.c_void_p()
        st = rt._lib.rt_scene_upload(C.byref(c), None, C.byref(h))
        assert st == rt.RT_ERR_INVALID_ARG and not h.value, (field, val)
    c = rt.rt_scene_desc.from_buffer_copy(d.c)
    c.sphere_geom = None
    assert rt._lib.rt_scene_upload(C.byref(c), None, C.byref(C.c_void_p())) == 1
    assert rt._lib.rt_scene_upload(None, None, C.byref(C.c_void_p())) == 1
    assert rt._lib.rt_scene_upload(C.byref(d.c), None, None) == 1
    assert "out is NULL" in rt.rt_last_error()


FAKE_SCENE = 0x10   # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("cam,W,H,D", [
    (Camera(fov_deg=0.0), 8, 8, 1), (Camera(fov_deg=180.0), 8, 8, 1),
    (Camera(eye=(0.0, float("nan"), 0.0)), 8, 8, 1), (Camera(yaw_deg=float("inf")), 8, 8, 1),
    (Camera(), 0, 8, 1), (Camera(), 8, -3, 1), (Camera(), 16385, 8, 1),
    (Camera(), 8, 8, -1), (Camera(), 8, 8, 9)])
def test_render_rejects_bad_camera_and_sizes(rt, cam, W, H, D):
    c = rt.make_camera(cam)
    st = rt._lib.rt_render(FAKE_SCENE, C.byref(c), W, H, D, 0x1000, None, None, None)
    assert st == rt.RT_ERR_INVALID_ARG
    st = rt._lib.rt_render_backward(FAKE_SCENE, C.byref(c), W, H, D, 0x1000, None,
                                    C.byref(rt.rt_grads()), None)
    assert st == rt.RT_ERR_INVALID_ARG
    st = rt._lib.rt_render_backward_static(FAKE_SCENE, C.byref(c), W, H, D, 0x1000, None,
                                           C.byref(rt.rt_grads()), None)
    assert st == rt.RT_ERR_INVALID_ARG


def test_render_rejects_null_buffers_and_short_records(rt):
    c = rt.make_camera(Camera())
    assert rt._lib.rt_render(None, C.byref(c), 8, 8, 1, 0x1000, None, None, None) == 1
    assert rt._lib.rt_render(FAKE_SCENE, C.byref(c), 8, 8, 1, None, None, None, None) == 1
    assert rt._lib.rt_render(FAKE_SCENE, None, 8, 8, 1, 0x1000, None, None, None) == 1
    rec = rt.rt_records(0x1000, 0x2000, rt.rt_records_bytes(8, 8, 1) - 1)
    assert rt._lib.rt_render(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, None, C.byref(rec),
                             None) == 1
    assert "records hold" in rt.rt_last_error()
    rec = rt.rt_records(None, 0x2000, 1 << 20)
    assert rt._lib.rt_render(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, None, C.byref(rec),
                             None) == 1
    assert rt._lib.rt_render_backward(FAKE_SCENE, C.byref(c), 8, 8, 1, None, None,
                                      C.byref(rt.rt_grads()), None) == 1
    assert rt._lib.rt_render_backward(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, None, None,
                                      None) == 1
    for f in (rt._lib.rt_render_backward_static,):
        assert f(None, C.byref(c), 8, 8, 1, 0x1000, None, C.byref(rt.rt_grads()), None) == 1
        assert f(FAKE_SCENE, C.byref(c), 8, 8, 1, None, None, C.byref(rt.rt_grads()), None) == 1
        assert f(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, None, None, None) == 1
    assert rt._lib.rt_render_counts(FAKE_SCENE, C.byref(c), 8, 8, 1, None, 0, None) == 1
    assert rt._lib.rt_render_counts(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, 2, None) == 1


def test_set_sky_rejects_bad_arguments_before_any_device_call(rt):
    sky = np.ones((4, 8, 3), np.float32)
    p = sky.ctypes.data
    f = rt._lib.rt_scene_set_sky
    assert f(None, p, 8, 4, 0, None) == rt.RT_ERR_INVALID_ARG
    for w, h in ((0, 4), (8, 0), (-1, 4), (rt.RT_MAX_SKY_DIM + 1, 1), (1, rt.RT_MAX_SKY_DIM + 1)):
        assert f(FAKE_SCENE, p, w, h, 0, None) == rt.RT_ERR_INVALID_ARG, (w, h)
    assert f(FAKE_SCENE, None, 8, 4, 0, None) == rt.RT_ERR_INVALID_ARG
    assert f(FAKE_SCENE, None, 0, 4, 0, None) == rt.RT_ERR_INVALID_ARG
    assert f(FAKE_SCENE, p, 8, 4, 7, None) == rt.RT_ERR_INVALID_ARG
    for bad in (np.nan, np.inf, -np.inf):
        s = sky.copy()
        s[3, 7, 2] = bad
        assert f(FAKE_SCENE, s.ctypes.data, 8, 4, 0, None) == rt.RT_ERR_INVALID_ARG
        assert "non-finite" in rt.rt_last_error()
    with pytest.raises(ValueError):
        rt.rt_scene_set_sky(FAKE_SCENE, np.ones((4, 8), np.float32))


def test_frame_rejects_bad_arguments_before_any_device_call(rt):
    good = dict(W=8, H=8, soft=0, stream_out=0, format=0, flags=0, rgb_out=0x1000)
    f = C.c_void_p()
    for field, val in (("W", 0), ("H", -1), ("W", rt.RT_MAX_DIM + 1), ("soft", 2), ("flags", 4),
                       ("rgb_out", None), ("format", 2), ("format", rt.RT_FRAME_ARGB8)):
        d = rt.rt_frame_desc(**{**good, field: val})
        assert rt._lib.rt_frame_create(FAKE_SCENE, C.byref(d), C.byref(f)) == 1, field
        assert not f.value
    d = rt.rt_frame_desc(**good)
    assert rt._lib.rt_frame_create(None, C.byref(d), C.byref(f)) == 1
    assert rt._lib.rt_frame_create(FAKE_SCENE, None, C.byref(f)) == 1
    assert rt._lib.rt_frame_create(FAKE_SCENE, C.byref(d), None) == 1
    inp = rt.rt_frame_input(rt.make_camera(Camera()), 1, 1, 0.0, None)
    assert rt._lib.rt_frame_submit(None, C.byref(inp), None) == 1
    assert rt._lib.rt_frame_submit(FAKE_SCENE, None, None) == 1
    assert rt._lib.rt_frame_result(None, None) == 1
    assert rt._lib.rt_frame_destroy(None) == 0


def test_batch_rejects_bad_arguments_before_any_device_call(rt):
    """rt_batch_create checks sizes, cameras and the total tile count before it
    reads a scene: placeholder scene and image pointers are never followed."""
    def create(n, W, H, depth=1, cam=Camera()):
        scenes = (C.c_void_p * n)(*([FAKE_SCENE] * n))
        cams = (rt.rt_camera * n)(*([rt.make_camera(cam)] * n))
        arr = lambda v: (C.c_int32 * n)(*([v] * n))
        outs = (C.c_void_p * n)(*([0x1000] * n))
        b = C.c_void_p(0x1234)
        st = rt._lib.rt_batch_create(n, scenes, cams, arr(W), arr(H), arr(depth), outs, 0, None,
                                     C.byref(b))
        assert not b.value
        return st
    assert create(0, 8, 8) == rt.RT_ERR_INVALID_ARG
    assert create(rt.RT_MAX_BATCH + 1, 8, 8) == rt.RT_ERR_INVALID_ARG
    assert create(2, rt.RT_MAX_DIM + 1, 8) == rt.RT_ERR_INVALID_ARG
    assert create(2, 8, 8, depth=rt.RT_MAX_DEPTH + 1) == rt.RT_ERR_INVALID_ARG
    assert create(2, 8, 8, cam=Camera(fov_deg=180.0)) == rt.RT_ERR_INVALID_ARG
    # every size at its maximum: 4096 x 16384^2 pixels make about 1.7e10
    # one-wave tiles, past the queue's 32-bit tile numbers
    assert create(rt.RT_MAX_BATCH, rt.RT_MAX_DIM, rt.RT_MAX_DIM) == rt.RT_ERR_INVALID_ARG
    assert "tiles" in rt.rt_last_error()


def test_destroy_null_is_a_no_op(rt):
    assert rt._lib.rt_scene_destroy(None) == 0


def test_build_script_loads_without_the_library():
    """__graft_entry__.build() must work on a fresh checkout, where the
    package (which needs the built library) cannot be imported yet: it loads
    the build script by path, and the script compiles every HIP source."""
    import subprocess
    import sys
    code = (
        "import sys, glob, os\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import __graft_entry__ as g\n"
        "b = g._load_hip_build()\n"
        "assert 'paper_2305_07450_amd' not in sys.modules\n"
        "srcs = sorted(os.path.basename(s) for s in b.sources())\n"
        f"want = sorted(os.path.basename(s) for s in glob.glob(os.path.join({ROOT!r}, 'paper_2305_07450_amd', 'csrc', '*.hip')))\n"
        "assert srcs == want and srcs, (srcs, want)\n"
        "assert '--offload-arch=gfx950' in b.FLAGS\n"
        "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.mark.parametrize("bad", ["cpu", "float64", "list"])
def test_binding_refuses_host_and_mistyped_buffers(rt, bad):
    """The binding checks every caller buffer (device, dtype, contiguity, size)
    before it calls the library: a host or float64 tensor never reaches a
    kernel as a device pointer."""
    import torch
    W, H, D = 8, 4, 1
    make = {"cpu": lambda *s: torch.zeros(*s, dtype=torch.float32),
            "float64": lambda *s: torch.zeros(*s, dtype=torch.float64),
            "list": lambda *s: [0.0] * int(np.prod(s))}[bad]
    cam = Camera()
    calls = [
        lambda: rt.rt_render(FAKE_SCENE, cam, W, H, D, make(H, W, 3)),
        lambda: rt.rt_render_ex(FAKE_SCENE, cam, W, H, D, make(H, W, 3), flags=0),
        lambda: rt.rt_render_soft(FAKE_SCENE, cam, W, H, D, 8, 0.5, make(H, W, 3)),
        lambda: rt.rt_render_counts(FAKE_SCENE, cam, W, H, D, make(7)),
        lambda: rt.rt_render_backward(FAKE_SCENE, cam, W, H, D, make(H, W, 3), {}),
        lambda: rt.rt_batch_create([FAKE_SCENE], [cam], [W], [H], [D], [make(H, W, 3)]),
        lambda: rt.rt_frame_create(FAKE_SCENE, W, H, make(H, W, 3)),
    ]
    for i, call in enumerate(calls):
        with pytest.raises(ValueError):
            call()


def test_binding_checks_scene_array_sizes(rt):
    s = scenegen.tiny_scene(1, n_spheres=3, n_lights=1)
    arrays = {k: getattr(s, k) for k in ("sphere_geom", "sphere_mat", "sphere_shine",
                                         "plane_geom", "plane_mat", "plane_shine", "light")}
    arrays["sphere_shine"] = arrays["sphere_shine"][:2]
    with pytest.raises(ValueError, match="sphere_shine"):
        rt._Desc(s, arrays)
    arrays = dict(arrays, sphere_shine=s.sphere_shine, sphere_geom=s.sphere_geom[:, :3])
    with pytest.raises(ValueError, match="sphere_geom"):
        rt._Desc(s, arrays)


def test_batch_tile_limit_boundary(rt):
    """The queue numbers tiles with 32-bit integers and hands out unsigned
    tickets up to n_tiles + grid - 1: 512 images of 16384 x 16384 make
    exactly 2^31 one-wave tiles, one past the limit, and are refused before
    any scene is read."""
    n = 512
    scenes = (C.c_void_p * n)(*([FAKE_SCENE] * n))
    cams = (rt.rt_camera * n)(*([rt.make_camera(Camera())] * n))
    arr = lambda v: (C.c_int32 * n)(*([v] * n))
    outs = (C.c_void_p * n)(*([0x1000] * n))
    b = C.c_void_p()
    st = rt._lib.rt_batch_create(n, scenes, cams, arr(rt.RT_MAX_DIM), arr(rt.RT_MAX_DIM), arr(1),
                                 outs, 0, None, C.byref(b))
    assert st == rt.RT_ERR_INVALID_ARG and not b.value
    assert "2147483648 tiles" in rt.rt_last_error()


def test_scene_counts_rejects_null(rt):
    assert rt._lib.rt_scene_counts(None, None, None, None) == rt.RT_ERR_INVALID_ARG


def test_prepare_and_flags_are_checked_on_the_host(rt):
    c = rt.make_camera(Camera())
    assert rt._lib.rt_render_prepare(None, C.byref(c), 8, 8, None) == rt.RT_ERR_INVALID_ARG
    assert rt._lib.rt_render_prepare(FAKE_SCENE, None, 8, 8, None) == rt.RT_ERR_INVALID_ARG
    bad = rt.make_camera(Camera(fov_deg=0.0))
    assert rt._lib.rt_render_prepare(FAKE_SCENE, C.byref(bad), 8, 8, None) == rt.RT_ERR_INVALID_ARG
    for W, H in ((0, 8), (8, 0), (rt.RT_MAX_DIM + 1, 8)):
        assert rt._lib.rt_render_prepare(FAKE_SCENE, C.byref(c), W, H, None) == rt.RT_ERR_INVALID_ARG
    assert rt._lib.rt_render_ex(FAKE_SCENE, C.byref(c), 8, 8, 1, 0x1000, None, None, 8,
                                None) == rt.RT_ERR_INVALID_ARG
    # soft renders and frames take no prepared cones
    assert rt._lib.rt_render_soft(FAKE_SCENE, C.byref(c), 8, 8, 1, 8, 0.5, 0x1000, None,
                                  rt.RT_RENDER_CONES_READY, None) == rt.RT_ERR_INVALID_ARG
