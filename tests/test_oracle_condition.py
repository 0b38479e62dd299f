"""Pins of the oracle's conditioning classifier, oracle.condition().

The colour bar of the GPU parity tests (1e-4 against the FP64 oracle) is
applied to pixels that condition() keeps: those whose decision record (hit
primitive and lit lights of every segment) survives K re-traces with each
segment's ray jittered by a few FP32 ulps, and whose colour spread over the
re-traces stays small.  Two pins fix what it must and must not exclude:

  * a lone diffuse sphere over a ground plane at depth 0 (primary hit, one
    light, a cast shadow): every pixel a few pixels away from a silhouette,
    the terminator or the shadow's edge is a smooth function of its ray, and
    must be kept;
  * a ray that bounces back and forth between two small mirror spheres: each
    bounce off a sphere of radius r after a flight of length t multiplies an
    angular error by about 1 + 2t/r (the curvature of a convex mirror), so
    four bounces turn ulp-sized jitter into a visibly different path, and the
    pixel must be excluded; the same pixel without the bounces is kept.

The per-workload excluded shares of the benchmark workloads are recorded by
tests/golden/condition_shares.json (written by the script beside it from the
oracle alone) and checked here for the small workload.
"""

import json
import os

import numpy as np
import pytest

import scenegen
from scenegen import Camera, Scene

F32 = np.float32
HERE = os.path.dirname(os.path.abspath(__file__))


def _scene(spheres, lights, planes, plane_mat, spec_strength=0.0):
    n = len(spheres)
    return Scene(
        sphere_geom=np.array([s[:4] for s in spheres], F32).reshape(n, 4),
        sphere_mat=np.array([s[4:8] for s in spheres], F32).reshape(n, 4),
        sphere_shine=np.full(n, 16, F32),
        plane_geom=np.array(planes, F32).reshape(-1, 4),
        plane_mat=np.array(plane_mat, F32).reshape(-1, 4),
        plane_shine=np.full(len(planes), 16, F32),
        light=np.array(lights, F32).reshape(-1, 4), spec_strength=spec_strength)


def test_lone_diffuse_sphere_is_well_conditioned_away_from_edges(oracle_mod):
    s = _scene([(0.0, 0.0, -4.5, 1.0, 0.6, 0.5, 0.4, 0.0)], [(4.0, 5.0, -2.0, 1.0)],
               scenegen.GROUND, [(0.7, 0.7, 0.7, 0.0)])
    cam = Camera(eye=(0.0, 1.0, 0.0), pitch_deg=-12.0)
    W, H = 96, 54
    base = oracle_mod.render(s, cam, W, H, 0)
    ok = oracle_mod.condition(s, cam, W, H, 0, base=base)
    # every discrete decision of the pixel in one key: the primary id and the
    # lit mask (n.L > 0 and no occluder: terminator and shadow edge)
    key = base.prim_id.astype(np.int64) * 4 + base.lit[:, 0]
    near_edge = oracle_mod.id_edges(key, W, H, radius=3)
    ids = base.prim_id
    assert (ids == 0).sum() > 300 and (ids == 1).sum() > 1000        # sphere and plane seen
    assert ((ids == 1) & (base.lit[:, 0] == 0)).sum() > 50           # a cast shadow seen
    assert ((ids == 0) & (base.lit[:, 0] == 0)).sum() > 50           # the unlit side seen
    bad = ~ok & ~near_edge
    assert not bad.any(), np.argwhere(bad.reshape(H, W))[:10]
    assert ok.mean() > 0.85


def _two_mirrors():
    # eye at the origin between sphere B (ahead, on -z) and sphere A (behind):
    # the centre pixel's ray runs along the axis joining them, hits B head-on,
    # comes back through the eye to A, and so on
    a = (0.0, 0.0, 2.0, 0.3, 0.5, 0.5, 0.5, 0.9)
    b = (0.0, 0.0, -2.5, 0.3, 0.5, 0.5, 0.5, 0.9)
    return _scene([a, b], [(1.5, 2.0, -0.5, 1.0)], np.zeros((0, 4)), np.zeros((0, 4)))


def test_bouncing_between_two_small_spheres_is_flagged(oracle_mod):
    s = _two_mirrors()
    W = H = 64
    pix = np.array([(H // 2) * W + W // 2])      # u = v = 0: the exact axis
    base = oracle_mod.render(s, Camera(), W, H, 4, pixels=pix)
    assert base.seg_id[0].tolist() == [1, 0, 1, 0, 1]
    assert not oracle_mod.condition(s, Camera(), W, H, 4, pixels=pix, base=base)[0]
    # without the bounces the same pixel is a plain diffuse hit: kept
    base0 = oracle_mod.render(s, Camera(), W, H, 0, pixels=pix)
    assert oracle_mod.condition(s, Camera(), W, H, 0, pixels=pix, base=base0)[0]


def test_jitter_is_the_only_source_of_exclusion_on_a_flat_scene(oracle_mod):
    """A plane-only scene lit from above has no silhouette, no occluder and no
    terminator in view: nothing may be excluded."""
    s = _scene([], [(0.0, 5.0, -5.0, 1.0)], scenegen.GROUND, [(0.3, 0.6, 0.9, 0.0)])
    cam = Camera(pitch_deg=-45.0)
    W, H = 64, 36
    assert oracle_mod.condition(s, cam, W, H, 2).all()


def test_recorded_shares_of_the_small_workload(oracle_mod):
    """The share of excluded pixels of the 256x144 workload equals the value
    the golden script recorded (the classifier has not drifted), under the
    settings the parity tests use."""
    with open(os.path.join(HERE, "golden", "condition_shares.json")) as f:
        g = json.load(f)
    rec = g["settings"]["current"]["workloads"]["fwd_256x144_8sph_1L_D2"]
    wl = scenegen.make_workload(0)
    ok = oracle_mod.condition(wl.scene, wl.camera, wl.W, wl.H, wl.depth)
    assert abs(float((~ok).mean()) - rec["ill_conditioned"]) < 1e-12
