"""Seeded synthetic inputs: Gaussian scenes and pinhole cameras.

This module only draws random numbers and builds camera poses. It holds none
of the method's arithmetic (no conversion, projection, binning or
compositing), so both the HIP path and the CPU oracle can take their inputs
from it.

Every array is produced in float64 and rounded once to float32; callers that
need float64 (the oracle) promote the float32 values back, so both sides see
the same numbers.

Layouts are structure-of-arrays with the component axis first:
  mean [3][N], scale [3][N] (linear, already activated), quat [4][N] as
  (w, x, y, z), opacity [N], rgb [3][N], sh [48][N] (basis-major,
  channel-minor: row = 3*basis + channel).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray      # [3][N] f32
    scale: np.ndarray     # [3][N] f32, linear
    quat: np.ndarray      # [4][N] f32, (w, x, y, z), unit length
    opacity: np.ndarray   # [N] f32 in (0, 1)
    rgb: np.ndarray       # [3][N] f32 in [0, 1]
    sh: np.ndarray | None = None  # [48][N] f32 or None

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])


@dataclasses.dataclass
class Camera:
    """OpenCV pinhole: x right, y down, z forward; pixel (i, j) centre at (i+0.5, j+0.5)."""
    world_to_cam: np.ndarray  # [3][4] f32, rows (R | t)
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.01


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def gaussians(n: int, seed: int, scale_lo: float, scale_hi: float, flat: bool,
              sh: bool = False) -> Gaussians:
    """Draws n Gaussians in a fixed order from default_rng(seed).

    Order: means U(-1, 1) (n,3); log-scales U(ln lo, ln hi) (n,3) -> exp, with
    the third column set to 0 for flat Gaussians; quaternions N(0, 1) (n,4)
    normalised, (w, x, y, z); opacity sigmoid(N(0, 1)); rgb U(0, 1) (n,3);
    optionally SH coefficients N(0, 0.1^2) (n,16,3).
    """
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, size=(n, 3))
    logs = rng.uniform(math.log(scale_lo), math.log(scale_hi), size=(n, 3))
    scale = np.exp(logs)
    if flat:
        scale[:, 2] = 0.0
    q = rng.standard_normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = 1.0 / (1.0 + np.exp(-rng.standard_normal(size=n)))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    shc = None
    if sh:
        shc = rng.normal(0.0, 0.1, size=(n, 16, 3)).reshape(n, 48)
    return Gaussians(mean=_f32(mean.T), scale=_f32(scale.T), quat=_f32(q.T),
                     opacity=_f32(op), rgb=_f32(rgb.T),
                     sh=None if shc is None else _f32(shc.T))


def look_at(center, width: int, height: int, fov_y_deg: float = 60.0,
            znear: float = 0.01) -> Camera:
    """Camera at `center` looking at the origin with world up +y.

    forward f = -c/|c|, right = normalize(f x up), down = f x right; focal
    length from the vertical field of view; principal point at the image centre.
    """
    c = np.asarray(center, dtype=np.float64)
    f = -c / np.linalg.norm(c)
    up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])            # rows: camera axes in world coordinates
    t = -R @ c
    w2c = np.concatenate([R, t[:, None]], axis=1)
    fy = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return Camera(world_to_cam=_f32(w2c), fx=float(np.float32(fy)), fy=float(np.float32(fy)),
                  cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                  width=int(width), height=int(height), znear=float(np.float32(znear)))


def ring_cameras(n_views: int, width: int, height: int, radius: float = 3.0,
                 elevation_deg: float = 0.0) -> list[Camera]:
    """Views on a horizontal ring: c_v = r (cos e sin phi, sin e, cos e cos phi), phi = 2 pi v / V."""
    cams = []
    e = math.radians(elevation_deg)
    for v in range(n_views):
        phi = 2.0 * math.pi * v / n_views
        c = radius * np.array([math.cos(e) * math.sin(phi), math.sin(e), math.cos(e) * math.cos(phi)])
        cams.append(look_at(c, width, height))
    return cams


def upstream_grad(n_views: int, height: int, width: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """dL/dimage, N(0, 1) * scale, layout [V][4][H][W] float32."""
    rng = np.random.default_rng(seed)
    return _f32(rng.standard_normal(size=(n_views, 4, height, width)) * scale)


def permuted(g: Gaussians, order) -> Gaussians:
    """The same scene with its Gaussians stored in `order` (e.g. the Morton order
    of their means), so that neighbouring Gaussians are near each other in
    memory; images do not depend on the storage order."""
    o = np.asarray(order, np.int64)
    return Gaussians(mean=_f32(g.mean[:, o]), scale=_f32(g.scale[:, o]), quat=_f32(g.quat[:, o]),
                     opacity=_f32(g.opacity[o]), rgb=_f32(g.rgb[:, o]), sh=None if g.sh is None else _f32(g.sh[:, o]))


def perturbed(g: Gaussians, seed: int) -> Gaussians:
    """Seeded perturbation of a scene, used to make fine-tuning targets:
    m += N(0, (0.25 s_max)^2); log s += N(0, 0.1^2) (zero scales stay zero);
    opacity logit += N(0, 0.25^2); rgb += N(0, 0.05^2) clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    mean = np.asarray(g.mean, np.float64)
    scale = np.asarray(g.scale, np.float64)
    n = mean.shape[1]
    smax = scale.max(axis=0)
    mean = mean + rng.normal(0, 1, (3, n)) * 0.25 * smax
    scale = scale * np.exp(rng.normal(0, 0.1, (3, n)))
    o = np.clip(np.asarray(g.opacity, np.float64), 1e-6, 1 - 1e-6)
    logit = np.log(o / (1 - o)) + rng.normal(0, 0.25, n)
    op = 1 / (1 + np.exp(-logit))
    rgb = np.clip(np.asarray(g.rgb, np.float64) + rng.normal(0, 0.05, (3, n)), 0, 1)
    return Gaussians(mean=_f32(mean), scale=_f32(scale), quat=g.quat.copy(), opacity=_f32(op), rgb=_f32(rgb),
                     sh=None if g.sh is None else g.sh.copy())


# ---------------------------------------------------------------------------
# The five workload shapes of the hot path (sizes as stated with the metric).
# ---------------------------------------------------------------------------

def config1(seed: int = 0):
    """1,000 flat Gaussians, K=8, sigma=2, one 128x128 view at distance 3."""
    g = gaussians(1000, seed, 0.01, 0.1, flat=True)
    return g, ring_cameras(1, 128, 128), dict(K=8, sigma=2.0)


def config2(seed: int = 0):
    """100k 3D Gaussians (scales log-U[0.005, 0.05]), K=8, one 800x800 view."""
    g = gaussians(100_000, seed, 0.005, 0.05, flat=False)
    return g, ring_cameras(1, 800, 800), dict(K=8, sigma=2.0)


def config3(seed: int = 0, n: int = 500_000, views: int = 8, width: int = 1920, height: int = 1080):
    """500k flat Gaussians, K=16, SH degree 3, eight 1920x1080 ring views."""
    g = gaussians(n, seed, 0.01, 0.1, flat=True, sh=True)
    return g, ring_cameras(views, width, height), dict(K=16, sigma=2.0)


def config5(seed: int = 0, n: int = 3_000_000, views: int = 16, width: int = 1920, height: int = 1080):
    """3M flat Gaussians, K=8, sixteen 1920x1080 ring views."""
    g = gaussians(n, seed, 0.01, 0.1, flat=True)
    return g, ring_cameras(views, width, height), dict(K=8, sigma=2.0)


# ---------------------------------------------------------------------------
# A geometry mesh for the mesh-prior mode: stands in for a mesh estimated by an
# external surface-reconstruction tool.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Mesh:
    pos: np.ndarray   # [3][Vm] f32
    idx: np.ndarray   # [3][Fm] i32, counter-clockwise seen from outside
    rgb: np.ndarray   # [3][Vm] f32 in [0, 1]

    @property
    def n_faces(self) -> int:
        return int(self.idx.shape[1])


def icosphere(level: int, seed: int, radius: float = 1.0, bump: float = 0.1) -> Mesh:
    """Icosahedron split `level` times into four (edge midpoints pushed to the
    sphere): 20 4^level faces, 10 4^level + 2 vertices. Each vertex is then
    moved radially by bump * radius * sin(3 u . p + phase) and coloured
    0.5 + 0.5 sin(4 w_c . p + phase_c), with u, w_c unit vectors and phases
    drawn from default_rng(seed)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    p = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5],
                  [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        key = np.sort(e, axis=1)
        uniq, inv = np.unique(key[:, 0] * (len(p) + 1) + key[:, 1], return_inverse=True)
        a, b = uniq // (len(p) + 1), uniq % (len(p) + 1)
        mid = p[a] + p[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = len(p) + inv.reshape(3, -1)                        # midpoints of edges (0,1), (1,2), (2,0)
        p = np.concatenate([p, mid])
        f = np.concatenate([np.stack([f[:, 0], m[0], m[2]], 1), np.stack([f[:, 1], m[1], m[0]], 1),
                            np.stack([f[:, 2], m[2], m[1]], 1), np.stack([m[0], m[1], m[2]], 1)])
    rng = np.random.default_rng(seed)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    w = rng.normal(size=(3, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    ph = rng.uniform(0, 2 * math.pi, size=4)
    r = radius * (1.0 + bump * np.sin(3.0 * p @ u + ph[0]))
    pos = p * r[:, None]
    rgb = 0.5 + 0.5 * np.sin(4.0 * p @ w.T + ph[1:])
    return Mesh(pos=_f32(pos.T), idx=np.ascontiguousarray(f.T.astype(np.int32)), rgb=_f32(rgb.T))


# ---------------------------------------------------------------------------
# Secondary rays (structure-of-arrays float32: origin [3][n], dir [3][n], t0 [n], t1 [n]).
# ---------------------------------------------------------------------------

def shadow_rays(n: int, seed: int, light=(0.0, 4.0, 0.0)):
    """Segments from points drawn U(-1, 1)^3 (the scene's extent) to a point
    light: dir = light - origin, t in (1e-4, 1)."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-1.0, 1.0, size=(3, n))
    d = np.asarray(light, np.float64).reshape(3, 1) - o
    return _f32(o), _f32(d), np.full(n, 1e-4, np.float32), np.ones(n, np.float32)


def scatter_rays(n: int, seed: int):
    """Incoherent rays: origins U(-1, 1)^3, directions N(0, 1)^3 (isotropic), t in (1e-4, inf)."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-1.0, 1.0, size=(3, n))
    d = rng.normal(size=(3, n))
    return _f32(o), _f32(d), np.full(n, 1e-4, np.float32), np.full(n, np.inf, np.float32)
