"""Pins of the FP64 oracle against what the paper and geometry fix.

None of these re-type the oracle's formulas: they use the paper's worked
example, closed forms derived from geometry (tangent cones, projected disks,
poles of spheres, mirror images), invariants (rotation, superposition, depth
invariance) and an independent brute force (mpmath / exact rationals).
"""

import json
import math
import os

import numpy as np
import pytest

import scenegen
from scenegen import Camera, Scene, SPEC_BLINN, SPEC_PHONG

from . import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def scene_of(spheres=(), planes=(), lights=(), mats=None, shine=None, pmat=None, pshine=None,
             ambient=0.1, ks=1.0, spec_model=SPEC_BLINN, bg=(0.0, 0.0, 0.0)):
    spheres = np.array(spheres, np.float32).reshape(-1, 4)
    planes = np.array(planes, np.float32).reshape(-1, 4)
    lights = np.array(lights, np.float32).reshape(-1, 4)
    N, P = spheres.shape[0], planes.shape[0]
    mats = np.array(mats if mats is not None else [[0.8, 0.5, 0.25, 0.0]] * N, np.float32)
    shine = np.array(shine if shine is not None else [16.0] * N, np.float32)
    pmat = np.array(pmat if pmat is not None else [[0.5, 0.75, 0.25, 0.0]] * P, np.float32)
    pshine = np.array(pshine if pshine is not None else [8.0] * P, np.float32)
    return Scene(spheres, mats.reshape(-1, 4), shine, planes, pmat.reshape(-1, 4), pshine,
                 lights, ambient=ambient, spec_strength=ks, spec_model=spec_model, background=bg)


def pix(W, x, y):
    return np.array([y * W + x], np.int64)


# ---------------------------------------------------------------- cameras

def test_ndc_worked_example(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "ndc_worked_example.json")))
    W, H = g["W"], g["H"]
    x, y = g["pixel"]
    o, d = oracle_mod.camera_rays(Camera(), W, H, pix(W, x, y))
    # the pixel sits on the viewport origin, so its ray is the optical axis
    assert o[0].tolist() == [0.0, 0.0, 0.0]
    assert d[0].tolist() == [0.0, 0.0, -1.0]


@pytest.mark.parametrize("W,H", [(256, 144), (1280, 720), (100, 200), (64, 64), (7, 3)])
@pytest.mark.parametrize("fov", [30.0, 60.0, 90.0, 120.0])
def test_fov_spans_shorter_side(oracle_mod, W, H, fov):
    """The edge of the viewport on the shorter side sits at half the field of
    view from the optical axis (camera distance 1/tan(fov/2), Section 3.2.1)."""
    if W >= H and W % 2 == 0:
        o, d = oracle_mod.camera_rays(Camera(fov_deg=fov), W, H, pix(W, W // 2, 0))
        assert d[0, 1] > 0 and abs(d[0, 0]) < 1e-15          # straight up from the axis
    elif H % 2 == 0:
        o, d = oracle_mod.camera_rays(Camera(fov_deg=fov), W, H, pix(W, 0, H // 2))
        assert d[0, 0] < 0 and abs(d[0, 1]) < 1e-15          # straight left
    else:
        pytest.skip("no pixel on the axis line")
    angle = math.degrees(math.acos(-d[0, 2]))
    assert abs(angle - fov / 2) < 1e-9


def test_fov_90_unit_distance(oracle_mod):
    """At 90 degrees b = 1: the top-centre ray of a landscape image is at 45 degrees."""
    o, d = oracle_mod.camera_rays(Camera(fov_deg=90.0), 200, 100, pix(200, 100, 0))
    assert abs(d[0, 1] + d[0, 2]) < 1e-15 and d[0, 1] > 0


def test_pixels_step_evenly_on_viewport(oracle_mod):
    """Along the centre row the tangent of the ray angle grows by the same
    step for each pixel: the viewport is a flat plane sampled uniformly."""
    W, H, fov = 320, 180, 60.0
    xs = np.arange(W)
    o, d = oracle_mod.camera_rays(Camera(fov_deg=fov), W, H, (H // 2) * W + xs)
    tan_az = d[:, 0] / -d[:, 2]
    step = np.diff(tan_az)
    assert np.allclose(step, step[0], rtol=1e-12, atol=0)
    # the shorter side (height, 180 px) spans tan(fov/2) each way
    assert abs(step[0] * H / 2 - math.tan(math.radians(fov / 2))) < 1e-12
    assert tan_az[W // 2] == 0.0


@pytest.mark.parametrize("yaw,pitch,expect", [
    (90.0, 0.0, (-1.0, 0.0, 0.0)),
    (-90.0, 0.0, (1.0, 0.0, 0.0)),
    (180.0, 0.0, (0.0, 0.0, 1.0)),
    (0.0, 90.0, (0.0, 1.0, 0.0)),
    (0.0, 30.0, (0.0, 0.5, -math.sqrt(3) / 2)),
    (90.0, 30.0, (-math.sqrt(3) / 2, 0.5, 0.0)),   # pitch applied before yaw
])
def test_yaw_pitch_axis(oracle_mod, yaw, pitch, expect):
    o, d = oracle_mod.camera_rays(Camera(yaw_deg=yaw, pitch_deg=pitch), 64, 36, pix(64, 32, 18))
    assert np.allclose(d[0], expect, atol=1e-12)


def _rot_y_minus90(v):
    # exact rotation by -90 degrees about +y: (x, y, z) -> (-z, y, x)
    return np.stack([-v[:, 2], v[:, 1], v[:, 0]], axis=1)


def test_yaw_equals_rotated_scene(oracle_mod):
    """Turning the camera by +90 degrees equals turning the world by -90."""
    s = scenegen.tiny_scene(3, n_spheres=6, n_lights=2)
    W, H, D = 80, 45, 2
    # place the scene to the left (-x) so that a camera turned by +90 sees it
    left = s.copy()
    left.sphere_geom[:, :3] = np.stack([s.sphere_geom[:, 2], s.sphere_geom[:, 1],
                                        -s.sphere_geom[:, 0]], 1)
    left.light[:, :3] = np.stack([s.light[:, 2], s.light[:, 1], -s.light[:, 0]], 1)
    left = Scene(**{k: getattr(left, k) for k in left.__dataclass_fields__})
    back = left.copy()
    back.sphere_geom[:, :3] = _rot_y_minus90(left.sphere_geom[:, :3].astype(np.float64))
    back.light[:, :3] = _rot_y_minus90(left.light[:, :3].astype(np.float64))
    assert np.array_equal(back.sphere_geom, s.sphere_geom)
    a = oracle_mod.render(left, Camera(yaw_deg=90.0), W, H, D)
    b = oracle_mod.render(s, Camera(), W, H, D)
    ok = (a.margin > 1e-9) & (b.margin > 1e-9)
    assert ok.mean() > 0.95
    assert np.array_equal(a.prim_id[ok], b.prim_id[ok])
    assert np.abs(a.rgb[ok] - b.rgb[ok]).max() < 1e-9


# ---------------------------------------------------------- intersections

def _lone_sphere_hits(oracle_mod, c, r, W=96, H=54, cam=Camera()):
    s = scene_of(spheres=[[*c, r]], lights=[[0, 10, 0, 1]])
    pixels = np.arange(W * H)
    o, d = oracle_mod.camera_rays(cam, W, H, pixels)
    ids, ts = oracle_mod.closest_hits(s, o, d)
    return s, o, d, ids, ts


@pytest.mark.parametrize("seed", range(6))
def test_silhouette_equals_tangent_cone(oracle_mod, seed):
    """A pixel hits a lone sphere iff its ray lies inside the tangent cone
    from the eye, and the hit distance is the near end of the chord."""
    rng = np.random.default_rng(seed)
    c = np.array([rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(-9, -4)], np.float32)
    r = np.float32(rng.uniform(0.5, 1.5))
    cam = Camera(yaw_deg=float(rng.uniform(-10, 10)), pitch_deg=float(rng.uniform(-10, 10)))
    s, o, d, ids, ts = _lone_sphere_hits(oracle_mod, c.astype(np.float64), float(r), 192, 108,
                                         cam=cam)
    c64, r64 = c.astype(np.float64), float(r)
    dist = np.linalg.norm(c64)
    cosang = d @ c64 / dist
    theta = np.arccos(np.clip(cosang, -1, 1))
    half = math.asin(r64 / dist)
    clear = np.abs(theta - half) > 1e-9
    inside = theta < half
    assert inside.sum() > 10 and (~inside).sum() > 10
    assert np.array_equal(ids[clear] == 0, inside[clear])
    # near end of the chord: |c| cos(theta) - sqrt(r^2 - |c|^2 sin^2(theta))
    h = inside & clear
    t_geo = dist * np.cos(theta[h]) - np.sqrt(r64 ** 2 - (dist * np.sin(theta[h])) ** 2)
    assert np.allclose(ts[h], t_geo, rtol=1e-9, atol=0)


@pytest.mark.parametrize("z0,r,fov", [(-8.0, 1.0, 60.0), (-5.0, 2.0, 90.0), (-20.0, 0.5, 30.0)])
def test_on_axis_projected_disk(oracle_mod, z0, r, fov):
    """An on-axis sphere projects to a disk of viewport radius
    b * r / sqrt(z0^2 - r^2), b = 1/tan(fov/2)."""
    W, H = 400, 200
    s, o, d, ids, ts = _lone_sphere_hits(oracle_mod, (0.0, 0.0, z0), r, W, H, Camera(fov_deg=fov))
    b = 1.0 / math.tan(math.radians(fov) / 2)
    rho = b * r / math.sqrt(z0 * z0 - r * r)
    ys, xs = np.divmod(np.arange(W * H), W)
    u = (2.0 * xs - W) / H
    v = (H - 2.0 * ys) / H
    rad = np.hypot(u, v)
    clear = np.abs(rad - rho) > 1e-9
    assert np.array_equal(ids[clear] == 0, (rad < rho)[clear])


def test_origin_inside_sphere_takes_far_root(oracle_mod):
    g = np.array([0.0, 0.0, 0.0, 2.0])
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        assert abs(oracle_mod.sphere_root([0, 0, 0], d, g, 1e-3) - 2.0) < 1e-15
        # off-centre origin: far end of the chord along d
        o = np.array([0.5, -0.25, 0.75])
        t = oracle_mod.sphere_root(o, d, g, 1e-3)
        p = o + t * d
        assert abs(np.linalg.norm(p) - 2.0) < 1e-12 and t > 0
        assert (p - o) @ d > 0


def test_t_min_excludes_the_start_point(oracle_mod):
    """A ray leaving a sphere's surface outwards finds nothing; inwards it
    finds the far side of the chord, 2 r cos(angle to the inward normal)."""
    r = 1.5
    g = np.array([1.0, 2.0, -3.0, r])
    rng = np.random.default_rng(1)
    for _ in range(20):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        p = g[:3] + r * nrm
        out = rng.normal(size=3)
        out /= np.linalg.norm(out)
        if out @ nrm < 0.05:
            out = -out if -out @ nrm > 0.05 else nrm
        assert oracle_mod.sphere_root(p, out, g, 1e-3) is None
        inward = -out
        t = oracle_mod.sphere_root(p, inward, g, 1e-3)
        assert abs(t - 2 * r * (out @ nrm)) < 1e-12


def test_plane_roots_exact(oracle_mod):
    from fractions import Fraction
    rng = np.random.default_rng(2)
    for _ in range(200):
        m = rng.normal(size=3)
        m /= np.linalg.norm(m)
        g = np.array([*m, rng.uniform(-3, 3)])
        o = rng.uniform(-5, 5, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t = oracle_mod.plane_root(o, d, g, 1e-3)
        exact = bf.plane_roots(o, d, g)
        if not exact or exact[0] <= Fraction(1e-3):
            assert t is None
        else:
            te = float(exact[0])
            # forward error bound of (h - m.o) / (m.d) evaluated in FP64
            den = abs(g[:3] @ d)
            bound = 16 * 2.0 ** -53 * (abs(g[3]) + np.abs(g[:3] * o).sum()
                                       + abs(te) * np.abs(g[:3] * d).sum()) / den
            assert t is not None and abs(t - te) <= bound
    # a ray parallel to the plane misses
    assert oracle_mod.plane_root([0, 0, 0], [1, 0, 0], [0, 1, 0, -1], 1e-3) is None


@pytest.mark.parametrize("seed", range(8))
def test_bruteforce_hit_lists(oracle_mod, seed):
    """Closest hits agree with mpmath/exact-rational hit lists on tiny scenes,
    for camera rays and for rays starting on and inside the primitives."""
    rng = np.random.default_rng(100 + seed)
    s = scenegen.tiny_scene(200 + seed, n_spheres=int(rng.integers(1, 4)), n_lights=1,
                            with_plane=bool(seed % 2 == 0))
    W, H = 32, 18
    o, d = oracle_mod.camera_rays(Camera(), W, H, np.arange(W * H))
    extra_o, extra_d = [], []
    for i in range(s.n_spheres):
        c, r = s.sphere_geom[i, :3].astype(np.float64), float(s.sphere_geom[i, 3])
        for _ in range(8):
            nrm = rng.normal(size=3)
            nrm /= np.linalg.norm(nrm)
            dd = rng.normal(size=3)
            dd /= np.linalg.norm(dd)
            extra_o += [c + r * nrm, c + 0.3 * r * nrm]
            extra_d += [dd, dd]
    if extra_o:
        o = np.concatenate([o, np.array(extra_o)])
        d = np.concatenate([d, np.array(extra_d)])
    ids, ts = oracle_mod.closest_hits(s, o, d)
    checked = 0
    for k in range(o.shape[0]):
        hits = bf.hit_list(s, o[k], d[k])
        if len(hits) >= 2 and abs(float(hits[1][0] - hits[0][0])) < 1e-9 * float(hits[0][0]):
            continue   # near-tie: the order is not a robust FP64 decision
        if hits and abs(float(hits[0][0]) - float(s.t_min)) < 1e-9:
            continue
        want_id = hits[0][1] if hits else -1
        assert ids[k] == want_id, (k, hits[:2], ids[k], ts[k])
        if hits:
            assert abs(ts[k] - float(hits[0][0])) <= 1e-10 * max(1.0, float(hits[0][0]))
        checked += 1
    assert checked > 0.95 * o.shape[0]


def test_ties_go_to_lower_id(oracle_mod):
    g = [0.0, 0.0, -6.0, 1.0]
    s = scene_of(spheres=[[3.0, 0, -6, 0.5], g, [0, 5, -6, 0.5], g, g], lights=[[0, 10, 0, 1]])
    o, d = oracle_mod.camera_rays(Camera(), 64, 36, np.arange(64 * 36))
    ids, ts = oracle_mod.closest_hits(s, o, d)
    assert set(np.unique(ids)) <= {-1, 0, 1, 2}
    assert (ids == 1).sum() > 20


# ---------------------------------------------------------------- shading

def _pole_scene(light, a=(0.8, 0.5, 0.25), ks=1.0, shine=16.0, spec_model=SPEC_BLINN,
                z0=-6.0, r=1.0):
    return scene_of(spheres=[[0.0, 0.0, z0, r]], lights=[light], mats=[[*a, 0.0]],
                    shine=[shine], ks=ks, spec_model=spec_model)


def _centre_pixel(oracle_mod, s, depth=0, W=64, H=36):
    return oracle_mod.render(s, Camera(), W, H, depth, pixels=pix(W, W // 2, H // 2))


def test_lambert_at_the_pole(oracle_mod):
    """Centre pixel hits the near pole p = (0, 0, z0 + r), normal +z, so with
    no specular term C = a (k_a + I cos(angle to the light))."""
    q = np.array([3.0, 4.0, 2.0])
    s = _pole_scene([*q, 0.75], ks=0.0)
    r = _centre_pixel(oracle_mod, s)
    p = np.array([0.0, 0.0, -5.0])
    cosl = (q - p)[2] / np.linalg.norm(q - p)
    a = np.array([0.8, 0.5, 0.25], np.float32).astype(np.float64)
    ka = float(np.float32(0.1))
    assert r.prim_id[0] == 0
    assert np.allclose(r.rgb[0], a * (ka + 0.75 * cosl), rtol=0, atol=1e-13)


@pytest.mark.parametrize("model", [SPEC_BLINN, SPEC_PHONG])
def test_specular_peak_on_axis(oracle_mod, model):
    """Light on the axis behind the camera: L = V = n at the pole, so the
    specular factor is 1 for both models: C = a (k_a + I) + I k_s."""
    s = _pole_scene([0.0, 0.0, 4.0, 0.5], ks=1.0, spec_model=model, shine=40.0)
    r = _centre_pixel(oracle_mod, s)
    a = np.array([0.8, 0.5, 0.25], np.float32).astype(np.float64)
    ka = float(np.float32(0.1))
    assert np.allclose(r.rgb[0], a * (ka + 0.5) + 0.5, rtol=0, atol=1e-13)


@pytest.mark.parametrize("theta_deg", [20.0, 45.0, 70.0])
def test_specular_off_axis(oracle_mod, theta_deg):
    """Light at angle theta from the pole normal (view along the normal):
    Blinn's halfway vector is at theta/2, so spec = cos(theta/2)^s; Phong's
    mirrored light is at theta on the other side, so spec = cos(theta)^s."""
    th = math.radians(theta_deg)
    p = np.array([0.0, 0.0, -5.0])
    q = p + 7.0 * np.array([math.sin(th), 0.0, math.cos(th)])
    q32 = q.astype(np.float32).astype(np.float64)
    th_eff = math.atan2(q32[0] - p[0], q32[2] - p[2])   # angle after FP32 rounding of q
    a = np.array([0.8, 0.5, 0.25], np.float32).astype(np.float64)
    ka = float(np.float32(0.1))
    for model, spec in ((SPEC_BLINN, math.cos(th_eff / 2) ** 24),
                        (SPEC_PHONG, math.cos(th_eff) ** 24)):
        s = _pole_scene([*q, 1.0], shine=24.0, spec_model=model)
        r = _centre_pixel(oracle_mod, s)
        want = a * (ka + math.cos(th_eff)) + spec
        assert np.allclose(r.rgb[0], want, rtol=0, atol=1e-12), (model, r.rgb[0], want)


def _shadow_scene(extra_light=None, occluder_y=3.0):
    lights = [[0.0, 8.0, -10.0, 1.0]] + ([extra_light] if extra_light else [])
    return scene_of(spheres=[[0.0, occluder_y, -10.0, 1.0]], planes=[[0, 1, 0, -1]],
                    lights=lights, pmat=[[0.5, 0.75, 0.25, 0.0]], pshine=[8.0])


def _pixel_hitting(oracle_mod, cam, W, H, target):
    """Pixel whose primary ray passes closest to a target point."""
    o, d = oracle_mod.camera_rays(cam, W, H, np.arange(W * H))
    to = target - o
    perp = np.linalg.norm(to - (to * d).sum(1, keepdims=True) * d, axis=1)
    return int(np.argmin(perp))


def test_shadowed_point_gets_ambient_only(oracle_mod):
    """A plane point straight below an occluding sphere, under the light,
    keeps only the ambient share of its colour (Section 3.6)."""
    s = _shadow_scene()
    W, H = 160, 90
    k = _pixel_hitting(oracle_mod, Camera(), W, H, np.array([0.0, -1.0, -10.0]))
    r = oracle_mod.render(s, Camera(), W, H, 0, pixels=np.array([k]))
    assert r.prim_id[0] == 1 and r.lit[0, 0] == 0
    ka = float(np.float32(0.1))
    assert np.array_equal(r.rgb[0], ka * np.array([0.5, 0.75, 0.25], np.float32).astype(np.float64))


def test_shadow_from_one_of_two_lights(oracle_mod):
    """Occluded from light 0 and lit by light 1: only light 1 adds diffuse
    and specular light (ambient counted once)."""
    q1 = np.array([6.0, 5.0, -4.0])
    s = _shadow_scene(extra_light=[*q1, 0.5])
    W, H = 160, 90
    k = _pixel_hitting(oracle_mod, Camera(), W, H, np.array([0.0, -1.0, -10.0]))
    r = oracle_mod.render(s, Camera(), W, H, 0, pixels=np.array([k]))
    assert r.prim_id[0] == 1 and r.lit[0, 0] == 0b10
    o, d = oracle_mod.camera_rays(Camera(), W, H, np.array([k]))
    t = (-1.0 - o[0, 1]) / d[0, 1]
    p = o[0] + t * d[0]
    L = (q1 - p) / np.linalg.norm(q1 - p)
    nl = L[1]
    Hh = L - d[0]
    spec = (Hh[1] / np.linalg.norm(Hh)) ** 8
    a = np.array([0.5, 0.75, 0.25], np.float32).astype(np.float64)
    ka = float(np.float32(0.1))
    assert np.allclose(r.rgb[0], a * (ka + 0.5 * nl) + 0.5 * spec, rtol=0, atol=1e-12)


def test_occluder_beyond_light_casts_no_shadow(oracle_mod):
    s = _shadow_scene(occluder_y=12.0)      # sphere above the light
    W, H = 160, 90
    k = _pixel_hitting(oracle_mod, Camera(), W, H, np.array([0.0, -1.0, -10.0]))
    r = oracle_mod.render(s, Camera(), W, H, 0, pixels=np.array([k]))
    assert r.prim_id[0] == 1 and r.lit[0, 0] == 1


@pytest.mark.parametrize("model", [SPEC_BLINN, SPEC_PHONG])
def test_two_light_superposition(oracle_mod, model):
    """At depth 0 each lit light adds its own diffuse and specular light:
    C(L1 + L2) = C(L1) + C(L2) - k_a a on every hit pixel (misses are black)."""
    s = scenegen.tiny_scene(7, n_spheres=5, n_lights=2, spec_model=model)
    s1, s2 = s.copy(), s.copy()
    s1.light = s.light[:1].copy()
    s2.light = s.light[1:].copy()
    s1 = Scene(**{k: getattr(s1, k) for k in s1.__dataclass_fields__})
    s2 = Scene(**{k: getattr(s2, k) for k in s2.__dataclass_fields__})
    W, H = 96, 54
    r12 = oracle_mod.render(s, Camera(), W, H, 0)
    r1 = oracle_mod.render(s1, Camera(), W, H, 0)
    r2 = oracle_mod.render(s2, Camera(), W, H, 0)
    ids = r12.prim_id
    hit = ids >= 0
    alb = np.concatenate([s.sphere_mat[:, :3], s.plane_mat[:, :3]]).astype(np.float64)
    ka = float(s.ambient)
    want = r1.rgb[hit] + r2.rgb[hit] - ka * alb[ids[hit]]
    assert np.allclose(r12.rgb[hit], want, rtol=0, atol=1e-12)
    assert np.all(r12.rgb[~hit] == 0)
    assert (r12.lit[:, 0] == (r1.lit[:, 0] | (r2.lit[:, 0] << 1))).all()


# ------------------------------------------------------------- reflections

def test_depth_invariance_without_reflectivity(oracle_mod):
    s = scenegen.tiny_scene(11, n_spheres=6, n_lights=2)
    s.sphere_mat[:, 3] = 0
    s.plane_mat[:, 3] = 0
    W, H = 64, 36
    base = oracle_mod.render(s, Camera(), W, H, 0).rgb
    for D in range(1, 5):
        assert np.array_equal(oracle_mod.render(s, Camera(), W, H, D).rgb, base)


def _above_plane_scene(seed, n=5):
    """Random spheres entirely above the ground plane y = -1."""
    s = scenegen.tiny_scene(seed, n_spheres=n, n_lights=1)
    g = s.sphere_geom
    g[:, 1] = np.maximum(g[:, 1], -1.0 + g[:, 3] + 0.05)
    s.plane_mat[:, 3] = 0.4
    return s


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_mirror_camera_identity(oracle_mod, seed):
    """A ray reflected off the ground plane y = h continues like a ray from
    the eye mirrored in the plane: for plane pixels, the first bounce's hit
    equals the primary hit of the mirrored camera (eye (0, 2h, 0), pixel row
    H - y) in the scene without the plane."""
    s = _above_plane_scene(seed)
    W, H, h = 96, 54, -1.0
    r = oracle_mod.render(s, Camera(), W, H, 1)
    no_plane = Scene(s.sphere_geom, s.sphere_mat, s.sphere_shine, np.zeros((0, 4)),
                     np.zeros((0, 4)), np.zeros(0), s.light)
    mirror = Camera(eye=(0.0, 2 * h, 0.0))
    ys, xs = np.divmod(np.arange(W * H), W)
    sel = (r.prim_id == s.n_spheres) & (ys >= 1)
    mp = (H - ys[sel]) * W + xs[sel]
    m = oracle_mod.render(no_plane, mirror, W, H, 0, pixels=mp)
    ok = m.margin > 1e-7
    assert sel.sum() > 500 and ok.mean() > 0.97
    assert np.array_equal(r.seg_id[sel, 1][ok], m.prim_id[ok])
    assert (m.prim_id[ok] >= 0).sum() > 20


def test_reflection_mix_is_shaded(oracle_mod):
    """Depth 1 on a plane pixel whose bounce sees a sphere:
    C = A (1 - kr) a + S + A kr C_refl, with C_refl the mirrored camera's
    depth-0 colour (no plane) and A, S solved from two depth-0 renders with
    different plane albedo."""
    s = _above_plane_scene(31)
    W, H, h = 96, 54, -1.0
    r1 = oracle_mod.render(s, Camera(), W, H, 1)
    r0 = oracle_mod.render(s, Camera(), W, H, 0)
    s2 = s.copy()
    s2.plane_mat[:, :3] = 0.0
    r0b = oracle_mod.render(s2, Camera(), W, H, 0)
    ys, xs = np.divmod(np.arange(W * H), W)
    sel = (r1.prim_id == s.n_spheres) & (r1.seg_id[:, 1] >= 0) & (ys >= 1)
    no_plane = Scene(s.sphere_geom, s.sphere_mat, s.sphere_shine, np.zeros((0, 4)),
                     np.zeros((0, 4)), np.zeros(0), s.light)
    m = oracle_mod.render(no_plane, Camera(eye=(0.0, 2 * h, 0.0)), W, H, 0,
                          pixels=(H - ys[sel]) * W + xs[sel])
    ok = (m.margin > 1e-7) & (m.prim_id == r1.seg_id[sel, 1])
    assert ok.sum() > 20
    a = s.plane_mat[0, :3].astype(np.float64)
    kr = float(s.plane_mat[0, 3])
    S = r0b.rgb[sel][:, 0]                           # zero albedo leaves S alone
    A = (r0.rgb[sel][:, 0] - S) / a[0]
    want = A[:, None] * (1 - kr) * a + S[:, None] + A[:, None] * kr * m.rgb
    assert np.allclose(r1.rgb[sel][ok], want[ok], rtol=0, atol=1e-11)


# ----------------------------------------------------- margins and counts

def test_margin_silhouette_and_gap(oracle_mod):
    W, H = 64, 36
    k = pix(W, W // 2, H // 2)
    # the optical axis passes 2^-20 outside a sphere's silhouette
    r = 1.0
    x0 = 1.0 + 2.0 ** -20
    s = scene_of(spheres=[[x0, 0.0, -10.0, r]], lights=[[0, 10, 0, 1]])
    m = oracle_mod.render(s, Camera(), W, H, 0, pixels=k)
    x0f = float(np.float32(x0))
    assert m.prim_id[0] == -1
    assert abs(m.margin[0] - (x0f - r) / 10.0) < 1e-15 and m.margin[0] < 1e-6
    # two spheres on the axis, front surfaces 0.5 apart: gap (t2 - t1) / t1
    s = scene_of(spheres=[[0, 0, -10.0, 1.0], [0, 0, -10.5, 1.0]], lights=[[0, 10, 0, 1]])
    m = oracle_mod.render(s, Camera(), W, H, 0, pixels=k)
    assert m.prim_id[0] == 0 and abs(m.margin[0] - 0.5 / 9.0) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_counts_and_records_match_bruteforce(oracle_mod, seed):
    """Algorithmic counters and per-segment records equal a brute-force
    path walk with exact/mpmath hit lists (tiny scenes, every pixel)."""
    s = scenegen.tiny_scene(300 + seed, n_spheres=3, n_lights=2)
    W, H, D = 16, 9, 2
    r = oracle_mod.render(s, Camera(), W, H, D)
    o_all, d_all = oracle_mod.camera_rays(Camera(), W, H, np.arange(W * H))
    N, P = s.n_spheres, s.n_planes
    cnt = dict(sphere_tests=0, plane_tests=0, primary_rays=W * H, reflection_rays=0,
               shadow_rays=0)
    for k in range(W * H):
        o, d = o_all[k], d_all[k]
        for level in range(D + 1):
            if level:
                cnt["reflection_rays"] += 1
            cnt["sphere_tests"] += N
            cnt["plane_tests"] += P
            hid, t = bf.closest(s, o, d)
            assert r.seg_id[k, level] == hid
            if hid < 0:
                break
            p = o + t * d
            if hid < N:
                n = (p - s.sphere_geom[hid, :3].astype(np.float64)) / float(s.sphere_geom[hid, 3])
            else:
                n = s.plane_geom[hid - N, :3].astype(np.float64)
            lit = 0
            for l in range(s.n_lights):
                q = s.light[l, :3].astype(np.float64)
                dist = np.linalg.norm(q - p)
                L = (q - p) / dist
                if n @ L <= 0:
                    continue
                cnt["shadow_rays"] += 1
                occ, tested = bf.first_occluder(s, p, L, dist)
                n_sph = min(tested, N)
                cnt["sphere_tests"] += n_sph
                cnt["plane_tests"] += tested - n_sph
                if not occ:
                    lit |= 1 << l
            assert r.lit[k, level] == lit
            d = d - 2 * (d @ n) * n       # mirror image of the incoming direction
            o = p
    assert r.counts == cnt


def test_miss_is_background(oracle_mod):
    s = scene_of(spheres=[[0, 50, -10, 1.0]], lights=[[0, 10, 0, 1]], bg=(0.25, 0.5, 0.125))
    r = oracle_mod.render(s, Camera(), 32, 18, 3)
    assert (r.prim_id == -1).all()
    assert np.array_equal(r.rgb, np.tile([0.25, 0.5, 0.125], (32 * 18, 1)))
    assert (r.seg_id[:, 1:] == -2).all()


def test_workload_generator_is_deterministic():
    a = scenegen.make_workload(0)
    b = scenegen.make_workload(0)
    assert a.scene.digest() == b.scene.digest()
    assert a.scene.sphere_geom.dtype == np.float32
    assert a.scene.n_spheres == 8 and a.W == 256 and a.H == 144 and a.depth == 2
    g = a.scene.sphere_geom
    assert (g[:, 0] >= -4).all() and (g[:, 0] <= 4).all() and (g[:, 3] >= 0.3).all()
    batch = scenegen.make_batch()
    assert len(batch) == 64
    ns = [w.scene.n_spheres for w in batch]
    assert min(ns) >= 4 and max(ns) <= 1024
