"""Seeded synthetic inputs for the splat renderer.

This module only draws random numbers and assembles arrays: point clouds,
spherical-harmonic coefficients, opacities, radii, pinhole cameras, target
images and request traces.  It contains none of the renderer's arithmetic
(no projection, no SH evaluation, no compositing), so both the FP64 CPU oracle
and the HIP path can consume exactly the same bytes.

Every array is drawn in float64 from ``numpy.random.default_rng`` and cast to
float32 once, so both sides read identical float32 inputs.

Shapes follow the paper's data model (Sec. 3.1): points P_i in R^3 and per-point
SH coefficients h_{i,lm} for l <= l_max (l_max = 2 in the paper's experiments,
Sec. 3.3), stored as ``sh[N][(l_max+1)^2][3]``.  The per-point opacity and the
world-space splat radius are extra per-point inputs of this renderer.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Camera", "Scene", "seed_rng", "fov_focal", "look_at_camera",
    "random_sphere_camera", "orbit_camera", "random_scene_uniform_cube",
    "cube4k_128px", "ball100k_8x400", "surface300k_4x800", "dynamic30x200k_1024x768", "serving_scenes",
    "serving_trace", "small_scene", "SH_COEFFS", "Request", "hybrid_clouds", "point_attributes",
    "sphere_masks", "disc_views",
]

SH_COEFFS = {0: 1, 1: 4, 2: 9, 3: 16}


@dataclasses.dataclass
class Camera:
    """Pinhole camera: x_cam = R @ P + t; pixel = (fx*x/z + cx, fy*y/z + cy).

    R is 3x3 row-major (world -> camera), t is 3.  Axes follow the OpenCV
    convention: +x right, +y down (image rows), +z forward.
    """
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.width = int(self.width)
        self.height = int(self.height)

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    xyz: np.ndarray       # [N][3] float32
    sh: np.ndarray        # [N][K][3] float32
    opacity: np.ndarray   # [N] float32 in (0, 1)
    radius: np.ndarray    # [N] float32, world units

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def sh_degree(self) -> int:
        k = int(self.sh.shape[1])
        return {v: d for d, v in SH_COEFFS.items()}[k]


def seed_rng(stream: int) -> np.random.Generator:
    """Generator of workload stream s (1-based): child s-1 of SeedSequence(0)."""
    return np.random.default_rng(np.random.SeedSequence(0, spawn_key=(stream - 1,)))


def fov_focal(width: int, fov_deg: float = 50.0) -> float:
    """Focal length in pixels for a horizontal field of view."""
    return (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)


def look_at_camera(center, width: int, height: int, fov_deg: float = 50.0) -> Camera:
    """Camera at ``center`` looking at the origin.

    Rows of R are (right, down, forward); up is +z unless the view direction is
    within ~8 degrees of it, in which case +y is used.
    """
    c = np.asarray(center, dtype=np.float64)
    f = -c / np.linalg.norm(c)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ c
    fx = fov_focal(width, fov_deg)
    return Camera(R, t, fx, fx, width / 2.0, height / 2.0, width, height)


def random_sphere_camera(rng: np.random.Generator, width: int, height: int,
                         dist: float = 3.0, fov_deg: float = 50.0) -> Camera:
    g = rng.standard_normal(3)
    return look_at_camera(dist * g / np.linalg.norm(g), width, height, fov_deg)


def orbit_camera(frame: int, frames: int, width: int, height: int,
                 dist: float = 3.0, elev_deg: float = 20.0) -> Camera:
    th = 2.0 * math.pi * frame / frames
    el = math.radians(elev_deg)
    c = dist * np.array([math.cos(th) * math.cos(el), math.sin(th) * math.cos(el), math.sin(el)])
    return look_at_camera(c, width, height)


def _sh(rng, n, k=9, std=0.3):
    return (std * rng.standard_normal((n, k, 3))).astype(np.float32)


def _opacity(rng, n):
    return (1.0 / (1.0 + np.exp(-rng.standard_normal(n)))).astype(np.float32)


def _ball(rng, n):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def random_scene_uniform_cube(rng, n, sh_degree=2, radius=0.02, sh_std=0.3) -> Scene:
    xyz = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    sh = _sh(rng, n, SH_COEFFS[sh_degree], sh_std)
    op = _opacity(rng, n)
    return Scene(xyz, sh, op, np.full(n, radius, np.float32))


def small_scene(seed: int, n: int, sh_degree: int = 2, radius: float = 0.02,
                extent: float = 1.0, sh_std: float = 0.3) -> Scene:
    """Tiny scene for brute-force checks (xyz uniform in [-extent, extent]^3)."""
    rng = np.random.default_rng(np.random.SeedSequence(1000 + seed))
    xyz = rng.uniform(-extent, extent, (n, 3)).astype(np.float32)
    sh = _sh(rng, n, SH_COEFFS[sh_degree], sh_std)
    op = _opacity(rng, n)
    return Scene(xyz, sh, op, np.full(n, radius, np.float32))


# ----------------------------------------------------------------------------
# Workload shapes (sizes follow the paper's scenes: tens to hundreds of
# thousands of points, 128^2 to 1080p views, 1 to 30 frames).
# ----------------------------------------------------------------------------

def cube4k_128px():
    """4096 points uniform in [-1,1]^3, SH degree 2 ~ N(0, 0.3), opacity
    sigmoid(N(0,1)), radius 0.02; one camera at distance 3 looking at the
    origin (R = I, t = (0,0,3)), fov 50 deg, 128x128."""
    rng = seed_rng(1)
    scene = random_scene_uniform_cube(rng, 4096)
    fx = fov_focal(128)
    cam = Camera(np.eye(3), [0.0, 0.0, 3.0], fx, fx, 64.0, 64.0, 128, 128)
    return scene, [cam]


def ball100k_8x400(n: int = 100_000, views: int = 8, size: int = 400):
    """100k points uniform in the unit ball; 8 random views on the radius-3
    sphere at 400x400; uniform random targets; a 256-point gradient subset."""
    rng = seed_rng(2)
    dirs = rng.standard_normal((n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    xyz = (dirs * r[:, None]).astype(np.float32)
    sh = _sh(rng, n)
    op = _opacity(rng, n)
    scene = Scene(xyz, sh, op, np.full(n, 0.02, np.float32))
    cams = [random_sphere_camera(rng, size, size) for _ in range(views)]
    targets = rng.random((views, size, size, 3)).astype(np.float32)
    subset = np.sort(rng.choice(n, size=min(256, n), replace=False)).astype(np.int64)
    return scene, cams, targets, subset


def _bumps(rng, k=20):
    a = rng.uniform(-0.5, 0.5, k)
    mu = rng.uniform(-1.0, 1.0, (k, 2))
    s = rng.uniform(0.1, 0.3, k)
    return a, mu, s


def _height(xy, bumps):
    a, mu, s = bumps
    d2 = ((xy[:, None, :] - mu[None, :, :]) ** 2).sum(-1)
    return (a[None, :] * np.exp(-d2 / (2.0 * s[None, :] ** 2))).sum(-1)


def _surface_scene(rng, n, frac_on_surface, bumps=None, jitter=0.01):
    xyz = rng.uniform(-1.0, 1.0, (n, 3))
    if bumps is None:
        bumps = _bumps(rng)
    m = int(round(frac_on_surface * n))
    noise = jitter * rng.standard_normal(m)
    xyz[:m, 2] = _height(xyz[:m, :2], bumps) + noise
    sh = _sh(rng, n)
    op = _opacity(rng, n)
    return Scene(xyz.astype(np.float32), sh, op, np.full(n, 0.02, np.float32)), bumps


def surface300k_4x800(n: int = 300_000, size: int = 800, views_per_step: int = 4, steps: int = 100):
    """300k points uniform in [-1,1]^3, the first 30% moved onto a random
    surface z = sum of 20 Gaussian bumps (+ N(0, 0.01^2)); SH degree 2;
    4 views per step at 800x800 for 100 steps."""
    rng = seed_rng(3)
    scene, bumps = _surface_scene(rng, n, 0.3)
    cams = [random_sphere_camera(rng, size, size) for _ in range(views_per_step * steps)]
    # ground-truth scene for training targets: every point on the same surface
    grng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(5,)))
    gt, _ = _surface_scene(grng, n, 1.0, bumps=bumps)
    return scene, cams, gt


def dynamic30x200k_1024x768(frames: int = 30, n: int = 200_000, width: int = 1024, height: int = 768):
    """30 frames of 200k points moved by a smooth sinusoidal displacement
    field; SH shared across frames; one orbit view per frame at 1024x768."""
    rng = seed_rng(4)
    base = _ball(rng, n)
    W = rng.standard_normal((3, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, 3)
    sh = _sh(rng, n)
    op = _opacity(rng, n)
    rad = np.full(n, 0.02, np.float32)
    scenes = []
    arg0 = 2.0 * math.pi * (base @ W.T)
    for t in range(frames):
        xyz = base + 0.1 * np.sin(arg0 + 2.0 * math.pi * t / frames + phi[None, :])
        scenes.append(Scene(xyz.astype(np.float32), sh, op, rad))
    cams = [orbit_camera(t, frames, width, height) for t in range(frames)]
    targets_rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(3, 1)))
    return scenes, cams, targets_rng


RESOLUTIONS = [(256, 256), (512, 512), (800, 800), (1280, 720), (1920, 1080)]


def serving_scenes(count: int = 16, scale: float = 1.0):
    """16 resident scenes with log-uniform point counts in [5e4, 5e5], each
    drawn with the surface generator under its own seed."""
    rng = seed_rng(5)
    ns = np.round(np.exp(rng.uniform(math.log(5e4), math.log(5e5), count)) * scale).astype(int)
    scenes = []
    for s, n in enumerate(ns):
        srng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(4, 100 + s)))
        sc, _ = _surface_scene(srng, int(n), 0.3)
        scenes.append(sc)
    return scenes


@dataclasses.dataclass
class Request:
    arrival: float         # seconds after trace start
    scene: int
    camera: Camera


def serving_trace(n_scenes: int = 16, rate: float = 200.0, duration: float = 60.0,
                  seed_key: int = 0, resolutions: Optional[List] = None) -> List[Request]:
    """Poisson arrivals with random scene, random pose on the radius-3 sphere
    and a resolution drawn uniformly from the five serving sizes."""
    rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(4, 200 + seed_key)))
    res = resolutions or RESOLUTIONS
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = int(rng.integers(n_scenes))
        w, h = res[int(rng.integers(len(res)))]
        out.append(Request(t, s, random_sphere_camera(rng, w, h)))
    return out


def hybrid_clouds():
    """Point sets for the hybrid coarse-to-fine update (Sec. 3.3, Alg. 1) and
    its neighbour search, each stressing one structure: a uniform box of 3000
    points, five tight clusters plus uniform clutter (2200), a set with many
    exact duplicates (500), a set flat along z (800) and 40 collinear points at
    unit spacing (every neighbour distance tied)."""
    rng = np.random.default_rng(11)
    uni = rng.random((3000, 3)) * [2, 1, 0.5]
    cl = np.concatenate([c + 0.03 * rng.standard_normal((400, 3)) for c in rng.random((5, 3))] +
                        [rng.random((200, 3))])
    dup = rng.random((500, 3))
    dup[::7] = dup[3]
    flat = rng.random((800, 3))
    flat[:, 2] = 0.25
    line = np.zeros((40, 3))
    line[:, 0] = np.arange(40)
    return {k: v.astype(np.float32) for k, v in
            {"uniform": uni, "clusters": cl, "duplicates": dup, "flat": flat, "line": line}.items()}


def point_attributes(n: int, sh_degree: int = 2, seed: int = 0):
    """Per-point SH coefficients [n, (l+1)^2, 3] (standard normal), opacity in
    [0, 1) and radius in [0.01, 0.03), float32."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, (sh_degree + 1) ** 2, 3)).astype(np.float32),
            rng.random(n).astype(np.float32), rng.uniform(0.01, 0.03, n).astype(np.float32))


def disc_views(k: int, size: int = 64, dist: float = 3.0, seed: int = 0) -> List[Camera]:
    """k cameras at distance `dist` from the origin, looking at it from random
    directions, square images of `size` pixels (fov 50 degrees)."""
    rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(6, seed)))
    cams = []
    for _ in range(k):
        v = rng.standard_normal(3)
        cams.append(look_at_camera(dist * v / np.linalg.norm(v), size, size))
    return cams


def sphere_masks(cams, radius: float):
    """Foreground masks (uint8 [H, W]) of a sphere of `radius` at the origin:
    pixel (c, r) is foreground when the ray from the camera centre through the
    pixel centre (c + 0.5, r + 0.5) meets the sphere, i.e. its angle to the
    direction of the origin is at most asin(radius / distance)."""
    out = []
    for cam in cams:
        R = np.asarray(cam.R, np.float64).reshape(3, 3)
        t = np.asarray(cam.t, np.float64)
        C = -R.T @ t                                      # camera centre in the world
        d = np.linalg.norm(C)
        xs = (np.arange(cam.width) + 0.5 - cam.cx) / cam.fx
        ys = (np.arange(cam.height) + 0.5 - cam.cy) / cam.fy
        X, Y = np.meshgrid(xs, ys)
        dirs = np.stack([X, Y, np.ones_like(X)], -1) @ R   # camera -> world directions (rows)
        dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
        cosang = dirs @ (-C / d)
        out.append((cosang >= np.sqrt(max(0.0, 1.0 - (radius / d) ** 2))).astype(np.uint8))
    return out
