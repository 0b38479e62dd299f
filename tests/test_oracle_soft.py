"""Pins of the oracle's soft shadows (the paper's Section 3.6.1: a spherical
light sampled at n points of its great circle facing the hit point, in the
sunflower arrangement, shading scaled by the unblocked share).

  * a light of radius 0 is a point light: the image equals the hard-shadow
    render (every sample is the light centre);
  * a point that sees the whole disk unblocked is shaded exactly as under a
    point light, and a disk hidden by an occluder leaves ambient light only;
  * a sphere centred on the segment from the hit point to the light blocks
    exactly the samples at disk radius below rho = dist tan(asin(r / D)), so
    the number blocked is the count of points with 2 R sqrt(i/n) < rho, which
    is ceil(n rho^2 / (4 R^2)) (the sunflower radius law, with its factor 2,
    and a disk perpendicular to the direction to the light);
  * an occluder whose silhouette halves the disk leaves about half the
    light (the golden-angle spread covers both halves evenly).
"""

import math

import numpy as np
import pytest

import scenegen
from scenegen import Camera, Scene

F32 = np.float32


def scene_with(spheres, lights, plane=True, spec_strength=0.0, ambient=0.1):
    """Scene with given spheres (cx, cy, cz, r, albedo) and lights (x, y, z, I)."""
    n = len(spheres)
    geom = np.array([s[:4] for s in spheres], F32).reshape(n, 4)
    mat = np.array([[s[4], s[4], s[4], 0.0] for s in spheres], F32).reshape(n, 4)
    planes = scenegen.GROUND if plane else np.zeros((0, 4), F32)
    return Scene(sphere_geom=geom, sphere_mat=mat, sphere_shine=np.full(n, 16, F32),
                 plane_geom=planes, plane_mat=np.array([[0.8, 0.6, 0.4, 0.0]], F32)[:len(planes)],
                 plane_shine=np.full(len(planes), 16, F32),
                 light=np.array(lights, F32).reshape(-1, 4),
                 ambient=F32(ambient), spec_strength=F32(spec_strength))


def pixel_of(cam, W, H, target):
    """Pixel whose primary ray passes closest to a world point."""
    import oracle
    o, d = oracle.camera_rays(cam, W, H, np.arange(W * H))
    v = np.asarray(target, float) - o
    t = (v * d).sum(1)
    miss = np.linalg.norm(v - t[:, None] * d, axis=1)
    return int(np.argmin(miss))


def plane_point(oracle_mod, cam, W, H, pix):
    o, d = oracle_mod.camera_rays(cam, W, H, np.array([pix]))
    t = (-1.0 - o[0, 1]) / d[0, 1]      # the ground plane y = -1
    return o[0] + t * d[0]


def test_radius_zero_is_point_light(oracle_mod):
    s = scenegen.tiny_scene(7, n_spheres=12, n_lights=3)
    cam = Camera(yaw_deg=4.0, pitch_deg=-6.0)
    W, H, D = 48, 27, 2
    hard = oracle_mod.render(s, cam, W, H, D)
    soft = oracle_mod.render(s, cam, W, H, D, samples=37, light_radius=0.0)
    np.testing.assert_allclose(soft.rgb, hard.rgb, rtol=0, atol=1e-12)
    assert (soft.lit == hard.lit).all() and (soft.seg_id == hard.seg_id).all()


def test_unblocked_disk_is_point_light(oracle_mod):
    # a lone sphere lit from the camera side: near the point facing the light
    # the whole disk is in view and above the tangent plane
    s = scene_with([(0.0, 0.0, -8.0, 1.5, 0.7)], [(0.0, 0.0, 2.0, 1.0)], plane=False,
                   spec_strength=1.0)
    cam = Camera()
    W, H = 64, 64
    pix = np.array([32 * W + 32, 31 * W + 32, 32 * W + 33])
    hard = oracle_mod.render(s, cam, W, H, 0, pixels=pix)
    soft = oracle_mod.render(s, cam, W, H, 0, pixels=pix, samples=200, light_radius=0.5)
    assert (hard.prim_id == 0).all()
    np.testing.assert_allclose(soft.rgb, hard.rgb, rtol=0, atol=1e-12)


def test_hidden_disk_leaves_ambient(oracle_mod):
    cam = Camera()
    W, H = 64, 36
    pix = pixel_of(cam, W, H, (0.0, -1.0, -10.0))
    p = plane_point(oracle_mod, cam, W, H, pix)
    q = p + np.array([0.0, 6.0, 0.0])
    occ = p + np.array([0.0, 3.0, 0.0])            # radius 1.5 hides a disk of radius 1
    s = scene_with([(*occ, 1.5, 0.5)], [(*q, 1.0)])
    r = oracle_mod.render(s, cam, W, H, 0, pixels=np.array([pix]), samples=200, light_radius=1.0)
    assert r.prim_id[0] == 1     # the plane
    expect = float(s.ambient) * s.plane_mat[0, :3].astype(float)
    np.testing.assert_allclose(r.rgb[0], expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,R,frac_target", [(200, 1.0, 50.5), (64, 0.7, 20.3), (300, 1.3, 141.7)])
def test_concentric_occluder_counts_sunflower_radii(oracle_mod, n, R, frac_target):
    cam = Camera()
    W, H = 64, 36
    pix = pixel_of(cam, W, H, (0.0, -1.0, -10.0))
    p = plane_point(oracle_mod, cam, W, H, pix)
    dist = 6.0
    q = p + np.array([0.0, dist, 0.0])
    # occluder on the axis at D from p whose shadow cone from p has radius rho
    # on the light's disk, with n rho^2 / (4 R^2) = frac_target (not an integer)
    rho = math.sqrt(frac_target * 4.0 * R * R / n)
    Do = 3.0
    ro = Do * math.sin(math.atan(rho / dist))
    occ = p + np.array([0.0, Do, 0.0])
    s = scene_with([(*occ, ro, 0.5)], [(*q, 1.0)])
    # the scene is FP32: recompute rho from the stored values
    g = s.sphere_geom[0].astype(float)
    qq = s.light[0, :3].astype(float)
    rho = np.linalg.norm(qq - p) * math.tan(math.asin(g[3] / np.linalg.norm(g[:3] - p)))
    blocked = math.ceil(n * rho * rho / (4.0 * R * R))
    r = oracle_mod.render(s, cam, W, H, 0, pixels=np.array([pix]), samples=n, light_radius=R)
    assert r.prim_id[0] == 1
    a = s.plane_mat[0, :3].astype(float)
    nl = (qq - p)[1] / np.linalg.norm(qq - p)
    vis = (r.rgb[0] / a - float(s.ambient)) / nl
    np.testing.assert_allclose(vis, (n - blocked) / n, rtol=0, atol=1e-9)


def test_half_disk_occluder_halves_light(oracle_mod):
    cam = Camera()
    W, H = 64, 36
    pix = pixel_of(cam, W, H, (0.0, -1.0, -10.0))
    p = plane_point(oracle_mod, cam, W, H, pix)
    q = p + np.array([0.0, 6.0, 0.0])
    # a huge sphere whose surface passes through the axis point 3 units up:
    # near the axis it acts as the half-space x < 0 there
    big = 1000.0
    occ = p + np.array([-big, 3.0, 0.0])
    s = scene_with([(*occ, big, 0.5)], [(*q, 1.0)])
    r = oracle_mod.render(s, cam, W, H, 0, pixels=np.array([pix]), samples=200, light_radius=1.0)
    assert r.prim_id[0] == 1
    a = s.plane_mat[0, :3].astype(float)
    qq = s.light[0, :3].astype(float)
    nl = (qq - p)[1] / np.linalg.norm(qq - p)
    vis = (r.rgb[0] / a - float(s.ambient)) / nl
    assert abs(vis[0] - 0.5) < 0.06, vis


def _angle_law_count(n, R, alpha, delta, law):
    """Samples blocked by the half-space m.x < m.p - delta (m at angle alpha
    from the disk's first axis towards its second, both horizontal here),
    counted by hand from the sunflower law: point i at radius 2 R sqrt(i/n)
    and angle theta(i) = i x 137.507 degrees, the golden angle as the paper
    prints it.  `law` names the intended law or a plausible mistake."""
    blocked = 0
    for i in range(n):
        r = 2.0 * R * math.sqrt(i / n)
        th = {"printed": math.radians(i * 137.507),
              "radians": i * 137.507,                      # degrees read as radians
              "flipped": -math.radians(i * 137.507)}.get(law, math.radians(i * 137.507))
        if law == "swapped":                              # the two disk axes swapped
            along = r * (math.sin(th) * math.cos(alpha) + math.cos(th) * math.sin(alpha))
        else:
            along = r * (math.cos(th) * math.cos(alpha) + math.sin(th) * math.sin(alpha))
        blocked += along < -delta
    return blocked


@pytest.mark.parametrize("n,alpha_deg,want", [(23, 330.0, 11), (16, 270.0, 7), (22, 215.0, 10)])
def test_golden_angle_law_exact_count(oracle_mod, n, alpha_deg, want):
    """The angle law theta(i) = i phi pinned by an exact count.  The light is
    straight above the shaded ground point p, so the disk of samples is
    horizontal, with first axis +x and second axis -z (the orthonormal basis
    of Duff et al. for the up direction).  A vertical occluding plane with
    horizontal normal m at angle alpha from the first axis, at distance delta
    from p on the far side, blocks exactly the samples s with m.(s - q) <
    -delta: the shadow ray from p runs from one side of the plane to the
    other.  The camera and p lie on the same side of the wall.  The count
    follows by hand from the printed golden angle; degrees read as radians, a
    flipped angle and swapped axes each give another count, so each would
    fail."""
    R, delta = 1.0, 0.15
    alpha = math.radians(alpha_deg)
    cam = Camera()
    W, H = 64, 36
    pix = pixel_of(cam, W, H, (0.0, -1.0, -10.0))
    p = plane_point(oracle_mod, cam, W, H, pix)
    q = p + np.array([0.0, 6.0, 0.0])
    # the disk axes for w = +y: e1 = +x, e2 = -z, so m in world coordinates
    # is cos(alpha) e1 + sin(alpha) e2
    m = np.array([math.cos(alpha), 0.0, -math.sin(alpha)])
    wall = [m[0], m[1], m[2], float(m @ p) - delta]
    s = scene_with([], [(*q, 1.0)], plane=False)
    s = Scene(sphere_geom=np.zeros((0, 4), F32), sphere_mat=np.zeros((0, 4), F32),
              sphere_shine=np.zeros(0, F32),
              plane_geom=np.array([scenegen.GROUND[0], wall], F32),
              plane_mat=np.array([[0.8, 0.6, 0.4, 0.0], [0.2, 0.2, 0.2, 0.0]], F32),
              plane_shine=np.full(2, 16, F32), light=s.light, ambient=s.ambient,
              spec_strength=F32(0.0))
    want_by_hand = _angle_law_count(n, R, alpha, delta, "printed")
    assert want_by_hand == want
    for wrong in ("radians", "flipped", "swapped"):
        assert _angle_law_count(n, R, alpha, delta, wrong) != want, wrong
    r = oracle_mod.render(s, cam, W, H, 0, pixels=np.array([pix]), samples=n, light_radius=R)
    assert r.prim_id[0] == 0     # the ground plane, seen in front of the wall
    a = s.plane_mat[0, :3].astype(float)
    qq = s.light[0, :3].astype(float)
    nl = (qq - p)[1] / np.linalg.norm(qq - p)
    vis = (r.rgb[0] / a - float(s.ambient)) / nl
    np.testing.assert_allclose(vis, (n - want) / n, rtol=0, atol=1e-9)
