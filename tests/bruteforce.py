"""Brute-force hit lists for tiny scenes, independent of the oracle's code.

Every primitive's roots are found from the unnormalised parametric form
|o + t d - c|^2 = r^2 written as a polynomial a t^2 + b t + c0 with
a = d.d (no unit-length assumption), solved with mpmath at 60 significant
digits; plane roots are exact rationals (fractions.Fraction) of the binary
inputs.  The closest hit is the smallest root above t_min over all
primitives, ties to the lower id.  Shadow occlusion and the algorithmic test
counts (first occluder in ascending id order) follow the same lists.
"""

from __future__ import annotations

from fractions import Fraction
from typing import List, Optional, Tuple

import mpmath
import numpy as np

mpmath.mp.dps = 60


def _mp(v):
    return [mpmath.mpf(float(x)) for x in v]


def sphere_roots(o, d, geom) -> List[mpmath.mpf]:
    o, d, g = _mp(o), _mp(d), _mp(geom)
    oc = [o[k] - g[k] for k in range(3)]
    a = sum(d[k] * d[k] for k in range(3))
    b = 2 * sum(d[k] * oc[k] for k in range(3))
    c0 = sum(oc[k] * oc[k] for k in range(3)) - g[3] * g[3]
    disc = b * b - 4 * a * c0
    if disc < 0:
        return []
    s = mpmath.sqrt(disc)
    return sorted([(-b - s) / (2 * a), (-b + s) / (2 * a)])


def plane_roots(o, d, geom) -> List[Fraction]:
    o = [Fraction(float(x)) for x in o]
    d = [Fraction(float(x)) for x in d]
    g = [Fraction(float(x)) for x in geom]
    den = sum(g[k] * d[k] for k in range(3))
    if den == 0:
        return []
    return [(g[3] - sum(g[k] * o[k] for k in range(3))) / den]


def hit_list(scene, o, d) -> List[Tuple[float, int]]:
    """All roots above t_min as (t, id), sorted by (t, id)."""
    t_min = mpmath.mpf(float(scene.t_min))
    out = []
    for i in range(scene.n_spheres):
        for t in sphere_roots(o, d, scene.sphere_geom[i]):
            if t > t_min:
                out.append((t, i))
                break
    for j in range(scene.n_planes):
        for t in plane_roots(o, d, scene.plane_geom[j]):
            if t > Fraction(float(scene.t_min)):
                out.append((mpmath.mpf(t.numerator) / t.denominator, scene.n_spheres + j))
    return sorted(out, key=lambda e: (e[0], e[1]))


def closest(scene, o, d) -> Tuple[int, Optional[float]]:
    hits = hit_list(scene, o, d)
    if not hits:
        return -1, None
    return hits[0][1], float(hits[0][0])


def first_occluder(scene, p, ldir, dist) -> Tuple[bool, int]:
    """(occluded, number of primitives tested before stopping) for a shadow
    ray scanned in ascending id order."""
    t_min = mpmath.mpf(float(scene.t_min))
    dist = mpmath.mpf(float(dist))
    n_total = scene.n_spheres + scene.n_planes
    for i in range(scene.n_spheres):
        for t in sphere_roots(p, ldir, scene.sphere_geom[i]):
            if t_min < t < dist:
                return True, i + 1
    for j in range(scene.n_planes):
        for t in plane_roots(p, ldir, scene.plane_geom[j]):
            tf = mpmath.mpf(t.numerator) / t.denominator
            if t_min < tf < dist:
                return True, scene.n_spheres + j + 1
    return False, n_total
