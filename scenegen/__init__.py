"""Seeded synthetic scenes and cameras for the Whitted ray-tracing workloads.

This module only draws random numbers and packs them into float32 arrays.  It
holds none of the rendering arithmetic, so both the FP64 oracle (test
infrastructure) and the HIP path consume exactly the same canonical FP32 scene
without sharing any code that computes an image.

Scene content follows the paper's object description (Section 3.4: every body
has a position, a size that is the radius for a sphere, a colour and a
reflectivity) with the reflectivity split into a specular exponent and a mix
ratio, and the paper's primitive set (spheres and planes).

Draw order for every scene (fixed, so that a seed names one scene):
sphere centres (N x 3) -> radii (N) -> albedo (N x 3) -> exponent
``integers(8, 65, N)`` -> reflection ratio kr (N) -> plane material (albedo 3,
exponent, kr) -> light positions (L x 3).  Light intensity is 1.0.
"""

from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Sequence, Tuple

import numpy as np

SPEC_BLINN = 0
SPEC_PHONG = 1

F32 = np.float32


def f32(x) -> float:
    """Round a Python number to the nearest float32 and return it as a float."""
    return float(np.float32(x))


@dataclasses.dataclass
class Scene:
    """Canonical FP32 scene.  Array layouts are the ones the C ABI takes."""

    sphere_geom: np.ndarray   # float32 [N, 4]: centre x y z, radius r
    sphere_mat: np.ndarray    # float32 [N, 4]: albedo r g b, reflection ratio kr
    sphere_shine: np.ndarray  # float32 [N]:    specular exponent s
    plane_geom: np.ndarray    # float32 [P, 4]: unit normal m x y z, offset h (m . x = h)
    plane_mat: np.ndarray     # float32 [P, 4]
    plane_shine: np.ndarray   # float32 [P]
    light: np.ndarray         # float32 [L, 4]: position x y z, intensity I
    ambient: float = f32(0.1)
    spec_strength: float = f32(1.0)
    t_min: float = f32(1e-3)
    background: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    spec_model: int = SPEC_BLINN

    def __post_init__(self):
        self.sphere_geom = np.ascontiguousarray(self.sphere_geom, dtype=F32).reshape(-1, 4)
        self.sphere_mat = np.ascontiguousarray(self.sphere_mat, dtype=F32).reshape(-1, 4)
        self.sphere_shine = np.ascontiguousarray(self.sphere_shine, dtype=F32).reshape(-1)
        self.plane_geom = np.ascontiguousarray(self.plane_geom, dtype=F32).reshape(-1, 4)
        self.plane_mat = np.ascontiguousarray(self.plane_mat, dtype=F32).reshape(-1, 4)
        self.plane_shine = np.ascontiguousarray(self.plane_shine, dtype=F32).reshape(-1)
        self.light = np.ascontiguousarray(self.light, dtype=F32).reshape(-1, 4)
        self.ambient = f32(self.ambient)
        self.spec_strength = f32(self.spec_strength)
        self.t_min = f32(self.t_min)
        self.background = tuple(f32(c) for c in self.background)
        self.spec_model = int(self.spec_model)

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_geom.shape[0])

    @property
    def n_planes(self) -> int:
        return int(self.plane_geom.shape[0])

    @property
    def n_lights(self) -> int:
        return int(self.light.shape[0])

    def copy(self) -> "Scene":
        return dataclasses.replace(
            self,
            sphere_geom=self.sphere_geom.copy(), sphere_mat=self.sphere_mat.copy(),
            sphere_shine=self.sphere_shine.copy(), plane_geom=self.plane_geom.copy(),
            plane_mat=self.plane_mat.copy(), plane_shine=self.plane_shine.copy(),
            light=self.light.copy())

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.sphere_geom, self.sphere_mat, self.sphere_shine, self.plane_geom,
                  self.plane_mat, self.plane_shine, self.light):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.array([self.ambient, self.spec_strength, self.t_min, *self.background],
                          dtype=F32).tobytes())
        h.update(bytes([self.spec_model]))
        return h.hexdigest()[:16]


@dataclasses.dataclass
class Camera:
    """Pinhole camera: eye position, yaw and pitch in degrees, field of view in degrees."""

    eye: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    yaw_deg: float = 0.0
    pitch_deg: float = 0.0
    fov_deg: float = 60.0

    def __post_init__(self):
        self.eye = tuple(f32(c) for c in self.eye)
        self.yaw_deg = f32(self.yaw_deg)
        self.pitch_deg = f32(self.pitch_deg)
        self.fov_deg = f32(self.fov_deg)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    camera: Camera
    W: int
    H: int
    depth: int


GROUND = np.array([[0.0, 1.0, 0.0, -1.0]], dtype=F32)   # the plane y = -1

BOX_SMALL = ((-4.0, -1.0, -12.0), (4.0, 2.0, -4.0))
BOX_MEDIUM = ((-10.0, -1.0, -30.0), (10.0, 4.0, -5.0))
BOX_LARGE = ((-20.0, -1.0, -60.0), (20.0, 6.0, -5.0))
LIGHT_BOX = ((-5.0, 4.0, -6.0), (5.0, 8.0, 0.0))
RADII_STD = (0.3, 1.0)
RADII_SMALL = (0.1, 0.6)


def random_scene(rng: np.random.Generator, n_spheres: int, n_lights: int,
                 box=BOX_SMALL, radii=RADII_STD, light_box=LIGHT_BOX,
                 planes: np.ndarray = GROUND, spec_model: int = SPEC_BLINN,
                 intensity: float = 1.0) -> Scene:
    """Draw one scene in the fixed order given in the module docstring."""
    lo, hi = np.array(box[0]), np.array(box[1])
    centres = rng.uniform(lo, hi, size=(n_spheres, 3))
    r = rng.uniform(radii[0], radii[1], size=n_spheres)
    albedo = rng.uniform(0.0, 1.0, size=(n_spheres, 3))
    shine = rng.integers(8, 65, size=n_spheres)
    kr = rng.uniform(0.0, 0.5, size=n_spheres)
    n_planes = int(np.asarray(planes).reshape(-1, 4).shape[0])
    p_albedo = rng.uniform(0.0, 1.0, size=(n_planes, 3)) if n_planes else np.zeros((0, 3))
    p_shine = rng.integers(8, 65, size=n_planes) if n_planes else np.zeros(0)
    p_kr = rng.uniform(0.0, 0.5, size=n_planes) if n_planes else np.zeros(0)
    llo, lhi = np.array(light_box[0]), np.array(light_box[1])
    lpos = rng.uniform(llo, lhi, size=(n_lights, 3))
    return Scene(
        sphere_geom=np.concatenate([centres, r[:, None]], axis=1),
        sphere_mat=np.concatenate([albedo, kr[:, None]], axis=1),
        sphere_shine=shine,
        plane_geom=np.asarray(planes, dtype=F32).reshape(-1, 4),
        plane_mat=np.concatenate([p_albedo, p_kr[:, None]], axis=1),
        plane_shine=p_shine,
        light=np.concatenate([lpos, np.full((n_lights, 1), intensity)], axis=1),
        spec_model=spec_model,
    )


# The five workloads.  Sizes: (W, H, spheres, lights, depth, sphere box, radii).
CONFIG_SHAPES = [
    dict(name="fwd_256x144_8sph_1L_D2", W=256, H=144, N=8, L=1, D=2, box=BOX_SMALL, radii=RADII_STD),
    dict(name="fwd_1920x1080_64sph_2L_D4", W=1920, H=1080, N=64, L=2, D=4, box=BOX_MEDIUM, radii=RADII_STD),
    dict(name="fwd_3840x2160_512sph_4L_D4", W=3840, H=2160, N=512, L=4, D=4, box=BOX_LARGE, radii=RADII_SMALL),
    dict(name="batch_64scenes", W=None, H=None, N=None, L=1, D=None, box=BOX_SMALL, radii=RADII_STD),
    dict(name="fwdbwd_1280x720_128sph_1L_D3", W=1280, H=720, N=128, L=1, D=3, box=BOX_MEDIUM, radii=RADII_STD),
]

CANONICAL_SEED_BASE = 1000
BATCH_RESOLUTIONS = [(320, 180), (640, 360), (1280, 720), (1920, 1080)]


def canonical_seed(config_index: int) -> int:
    return CANONICAL_SEED_BASE + config_index


def make_workload(config_index: int, seed: int | None = None) -> Workload:
    """Single-scene workloads 0, 1, 2 and 4 (the forward part of 4)."""
    if config_index == 3:
        raise ValueError("workload 3 is a batch: use make_batch()")
    c = CONFIG_SHAPES[config_index]
    seed = canonical_seed(config_index) if seed is None else seed
    rng = np.random.default_rng(seed)
    scene = random_scene(rng, c["N"], c["L"], box=c["box"], radii=c["radii"])
    return Workload(c["name"], scene, Camera(), c["W"], c["H"], c["D"])


def make_batch(seed: int | None = None, n_scenes: int = 64) -> List[Workload]:
    """Batch workload: per scene N = round(exp(U[ln 4, ln 1024])), a resolution
    from BATCH_RESOLUTIONS, depth U{1..4}, one light, small box and standard radii.
    Per-scene sub-seeds come from a master generator."""
    seed = canonical_seed(3) if seed is None else seed
    master = np.random.default_rng(seed)
    out = []
    for i in range(n_scenes):
        n = int(round(math.exp(master.uniform(math.log(4), math.log(1024)))))
        W, H = BATCH_RESOLUTIONS[int(master.integers(0, len(BATCH_RESOLUTIONS)))]
        depth = int(master.integers(1, 5))
        sub = int(master.integers(0, 2**31 - 1))
        scene = random_scene(np.random.default_rng(sub), n, 1, box=BOX_SMALL, radii=RADII_STD)
        out.append(Workload(f"batch{i}_{W}x{H}_{n}sph_D{depth}", scene, Camera(), W, H, depth))
    return out


@dataclasses.dataclass
class DiffProblem:
    """Differentiable workload: a scene, the same scene with perturbed parameters
    (rendered to make the target image), and the render settings."""

    workload: Workload
    target_scene: Scene


def perturb_scene(scene: Scene, rng: np.random.Generator, sigma: float = 0.05) -> Scene:
    """Perturb every differentiated parameter by N(0, sigma): albedo, kr, sphere
    centres, light position and intensity; clip albedo and kr to [0, 1] and I to >= 0."""
    t = scene.copy()
    N, L = scene.n_spheres, scene.n_lights
    t.sphere_mat[:, :3] = np.clip(t.sphere_mat[:, :3] + rng.normal(0, sigma, (N, 3)), 0, 1)
    t.sphere_mat[:, 3] = np.clip(t.sphere_mat[:, 3] + rng.normal(0, sigma, N), 0, 1)
    t.sphere_geom[:, :3] = t.sphere_geom[:, :3] + rng.normal(0, sigma, (N, 3))
    t.light[:, :3] = t.light[:, :3] + rng.normal(0, sigma, (L, 3))
    t.light[:, 3] = np.maximum(t.light[:, 3] + rng.normal(0, sigma, L), 0)
    return Scene(**{f.name: getattr(t, f.name) for f in dataclasses.fields(Scene)})


def make_diff_problem(seed: int | None = None, W: int = 1280, H: int = 720, N: int = 128,
                      depth: int = 3) -> DiffProblem:
    seed = canonical_seed(4) if seed is None else seed
    wl = make_workload(4, seed)
    if (W, H, N, depth) != (1280, 720, 128, 3):
        rng = np.random.default_rng(seed)
        scene = random_scene(rng, N, 1, box=BOX_MEDIUM, radii=RADII_STD)
        wl = Workload(f"fwdbwd_{W}x{H}_{N}sph_1L_D{depth}", scene, Camera(), W, H, depth)
    target = perturb_scene(wl.scene, np.random.default_rng(seed + 7919))
    return DiffProblem(wl, target)


# The paper's benchmark scene has one light, one plane and five spheres whose
# coordinates it does not print; this seeded stand-in draws five spheres of
# radius 0.5-1.0 in front of the camera above the ground plane and one light
# in the usual light box.  PAPER_LIGHT_RADIUS is the radius its soft shadows
# use (the paper does not give the light's size).
PAPER_BOX = ((-3.0, -0.5, -10.0), (3.0, 1.5, -4.0))
PAPER_RADII = (0.5, 1.0)
PAPER_LIGHT_RADIUS = 0.5
PAPER_SETTINGS = {"hard_1bounce": (1, 1), "soft200_3bounces": (200, 3)}   # (samples, depth)


def sky_map(seed: int = 38, w: int = 512, h: int = 256) -> np.ndarray:
    """Procedural equirectangular sky, float32 [h, w, 3], standing in for the
    paper's HDR skybox image: a vertical gradient (light at the horizon,
    deeper blue overhead, dark ground below), a bright sun about 5 degrees
    across and seeded low-frequency variation, all smooth over several texels."""
    rng = np.random.default_rng(seed)
    v = (np.arange(h) + 0.5) / h                 # 0 at the top
    u = (np.arange(w) + 0.5) / w
    lat = (0.5 - v)[:, None] * np.pi             # +pi/2 overhead
    lon = (u - 0.5)[None, :] * 2 * np.pi
    up = np.clip(np.sin(lat), -1, 1)
    sky = np.where(up[..., None] >= 0,
                   np.array([0.55, 0.70, 0.95]) * (1 - up[..., None]) ** 2
                   + np.array([0.10, 0.25, 0.70]) * (1 - (1 - up[..., None]) ** 2),
                   np.array([0.25, 0.22, 0.20]) * (1 + up[..., None]))
    sky = np.broadcast_to(sky, (h, w, 3)).copy()
    ph = rng.uniform(0, 2 * np.pi, size=(3, 2))
    for k, (a, b) in enumerate(ph):
        sky += 0.04 * (np.sin((k + 1) * lon + a) * np.cos((k + 2) * lat + b))[..., None]
    s_lon, s_lat = rng.uniform(-0.6, 0.6), rng.uniform(0.35, 0.7)
    cosang = (np.cos(lat) * np.cos(s_lat) * np.cos(lon - s_lon) + np.sin(lat) * np.sin(s_lat))
    sky += 2.0 * np.exp((cosang - 1.0) / 0.004)[..., None] * np.array([1.0, 0.95, 0.85])
    return np.clip(sky, 0.0, None).astype(F32)


def verlet_motion(scene: Scene, frames: int, seed: int = 7, dt: float = 1.0 / 60.0,
                  gravity: float = 9.81, speed: float = 2.0) -> np.ndarray:
    """Sphere centres for `frames` frames, float32 [frames, N, 3]: the paper's
    physics system moves its bodies by Verlet integration, and this stands in
    for it as a driver of the per-frame position stream.  Position Verlet,
    x_{k+1} = 2 x_k - x_{k-1} + a dt^2 with a = (0, -gravity, 0), from seeded
    initial velocities of magnitude up to `speed`; a sphere that sinks into
    the ground plane y = -1 is mirrored back above it (an elastic bounce;
    one that starts sunk bounces at its starting height).
    Frame 0 is the scene's own centres.  Host-side input generation only."""
    rng = np.random.default_rng(seed)
    g = np.asarray(scene.sphere_geom, dtype=np.float64).reshape(-1, 4)
    x = g[:, :3].copy()
    r = g[:, 3]
    v = rng.uniform(-speed, speed, size=x.shape)
    prev = x - v * dt
    acc = np.array([0.0, -gravity, 0.0])
    out = np.empty((frames, x.shape[0], 3), dtype=F32)
    floor = np.minimum(-1.0 + r, x[:, 1])    # a sphere that starts sunk bounces there
    for k in range(frames):
        out[k] = x.astype(F32)
        nxt = 2.0 * x - prev + acc * dt * dt
        low = nxt[:, 1] < floor
        # mirror both the new and the current height about the floor: the
        # vertical velocity changes sign, the horizontal one stays
        nxt[low, 1] = 2.0 * floor[low] - nxt[low, 1]
        x_c = x.copy()
        x_c[low, 1] = 2.0 * floor[low] - x[low, 1]
        prev, x = x_c, nxt
    return out


def paper_scene(seed: int = 2305) -> Scene:
    return random_scene(np.random.default_rng(seed), 5, 1, box=PAPER_BOX, radii=PAPER_RADII)


def tiny_scene(seed: int, n_spheres: int = 3, n_lights: int = 1, with_plane: bool = True,
               spec_model: int = SPEC_BLINN) -> Scene:
    """Small random scene for brute-force and edge-case tests."""
    rng = np.random.default_rng(seed)
    planes = GROUND if with_plane else np.zeros((0, 4), dtype=F32)
    return random_scene(rng, n_spheres, n_lights, box=BOX_SMALL, radii=RADII_STD,
                        planes=planes, spec_model=spec_model)
