"""Pins of the oracle's skybox (the paper's Section 3.8: a panoramic image
behind the scene, looked up by UV mapping on every miss).

  * a constant map is the background colour;
  * a "coordinate" map, whose texel (i, j) holds ((i + 1/2)/w, (j + 1/2)/h, 0),
    is linear, so bilinear filtering returns (u, v) itself: looking straight
    ahead gives (1/2, 1/2); yaw 90 degrees (facing -x) gives u = 1/4; pitch
    30 degrees up gives v = 1/3; yaw -120 and pitch -45 give (5/6, 3/4);
  * a mirror floor (reflection ratio 1, no lights) shows the sky reflected
    about the horizon: pitch -30 degrees sees v' = 1/3, scaled by the ambient
    term of the mirror.
"""

import numpy as np
import pytest

import scenegen
from scenegen import Camera, Scene

F32 = np.float32


def coord_map(w=360, h=180):
    i = (np.arange(w) + 0.5) / w
    j = (np.arange(h) + 0.5) / h
    m = np.zeros((h, w, 3))
    m[..., 0] = i[None, :]
    m[..., 1] = j[:, None]
    return m


def empty_scene():
    z4 = np.zeros((0, 4), F32)
    z1 = np.zeros(0, F32)
    return Scene(sphere_geom=z4, sphere_mat=z4, sphere_shine=z1, plane_geom=z4, plane_mat=z4,
                 plane_shine=z1, light=z4)


def test_constant_sky_is_background(oracle_mod):
    s = scenegen.tiny_scene(12, n_spheres=8, n_lights=2)
    cam = Camera(pitch_deg=-10.0)
    c = np.array([0.3, 0.5, 0.7], F32).astype(float)
    sky = np.broadcast_to(c, (16, 32, 3)).copy()
    a = oracle_mod.render(s, cam, 48, 27, 2, sky=sky)
    s_bg = Scene(**{**s.__dict__, "background": tuple(float(v) for v in c)})
    b = oracle_mod.render(s_bg, cam, 48, 27, 2)
    np.testing.assert_allclose(a.rgb, b.rgb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("yaw,pitch,u,v", [(0.0, 0.0, 0.5, 0.5), (90.0, 0.0, 0.25, 0.5),
                                           (0.0, 30.0, 0.5, 1.0 / 3.0),
                                           (-120.0, -45.0, 5.0 / 6.0, 0.75)])
def test_uv_mapping_of_view_directions(oracle_mod, yaw, pitch, u, v):
    W, H = 64, 36                      # the centre pixel looks straight along the view axis
    r = oracle_mod.render(empty_scene(), Camera(yaw_deg=yaw, pitch_deg=pitch), W, H, 0,
                          pixels=np.array([(H // 2) * W + W // 2]), sky=coord_map())
    np.testing.assert_allclose(r.rgb[0], [u, v, 0.0], rtol=0, atol=1e-12)


def test_mirror_floor_reflects_the_sky(oracle_mod):
    z4 = np.zeros((0, 4), F32)
    s = Scene(sphere_geom=z4, sphere_mat=z4, sphere_shine=np.zeros(0, F32),
              plane_geom=scenegen.GROUND, plane_mat=np.array([[0.9, 0.2, 0.4, 1.0]], F32),
              plane_shine=np.array([16], F32), light=z4)
    W, H = 64, 36
    r = oracle_mod.render(s, Camera(pitch_deg=-30.0), W, H, 1,
                          pixels=np.array([(H // 2) * W + W // 2]), sky=coord_map())
    assert r.prim_id[0] == 0                   # the plane
    ka = float(s.ambient)
    np.testing.assert_allclose(r.rgb[0], [ka * 0.5, ka / 3.0, 0.0], rtol=0, atol=1e-12)


def test_seam_wraps_around(oracle_mod):
    """Looking along +z puts u at 1, on the seam: x = w - 1/2 falls halfway
    between the last column and, wrapped around, the first, so the
    coordinate map gives (w - 1/2 + 1/2) / (2 w) = 1/2 in red.  Clamping
    instead of wrapping would give (w - 1/2) / w."""
    W, H = 64, 36
    m = coord_map(w=360, h=180)
    r = oracle_mod.render(empty_scene(), Camera(yaw_deg=180.0), W, H, 0,
                          pixels=np.array([(H // 2) * W + W // 2]), sky=m)
    np.testing.assert_allclose(r.rgb[0], [0.5, 0.5, 0.0], rtol=0, atol=1e-9)


def test_pole_clamps_to_the_top_row(oracle_mod):
    """Near straight up, y = v h - 1/2 < 0 lies above the first row's centre:
    both bilinear rows clamp to row 0, so green is that row's value 1/(2 h)
    exactly, where extrapolating would give less."""
    W, H = 64, 36
    h = 180
    r = oracle_mod.render(empty_scene(), Camera(pitch_deg=89.9), W, H, 0,
                          pixels=np.array([(H // 2) * W + W // 2]), sky=coord_map(w=360, h=h))
    np.testing.assert_allclose(r.rgb[0, 1], 0.5 / h, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r.rgb[0, 0], 0.5, rtol=0, atol=1e-9)
