"""Seeded synthetic scenes and cameras for the linear-primitive rasterizer.

This module only *draws inputs*: primitive parameters, pinhole cameras and
loss gradients.  It holds none of the rendering arithmetic, so the FP64
oracle and the HIP path can both consume it without sharing any of the
method's code.

The paper renders trained ScanNet++ and Mip-NeRF 360 captures (Sec. 4 and
App. A); those are not available, so the scenes below stand in for them with
the primitive counts, size distributions, opacity distributions, SH degree
and image sizes of the workloads that are measured.  All draws come from
``numpy.random.default_rng(seed)`` (PCG64) in the order written here and are
returned as float32, which is the precision the primitives are stored in
(Sec. 3.1, "Memory Requirements": 11/12 floats plus 48 SH coefficients).

Primitive parameters follow the paper's parameterisation (Sec. 3.1):
  * ``means``   [N,3]  primitive centre
  * ``quats``   [N,4]  rotation quaternion (w, x, y, z), not necessarily unit
  * ``dists``   [N,3] (octahedron, one distance per pair of opposite vertices)
                [N,4] (tetrahedron, one distance per corner)
  * ``opacity`` [N]    activated opacity alpha in [0, 1]
  * ``sh``      [N,16,3] SH coefficients, coefficient-major, RGB last
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

OCTAHEDRON = 0
TETRAHEDRON = 1
NEAR_Z = 0.2


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward)."""

    world_to_cam: np.ndarray  # [3,4] float32, row-major [R | t]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = NEAR_Z

    def as_row(self) -> np.ndarray:
        """The 20 numbers of the camera, each rounded to float32 first."""
        v = np.zeros(20, dtype=np.float64)
        v[:12] = self.world_to_cam.astype(np.float32).reshape(-1)
        v[12:16] = np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)
        v[16] = self.width
        v[17] = self.height
        v[18] = np.float32(self.near)
        return v


@dataclasses.dataclass
class Scene:
    kind: int  # OCTAHEDRON or TETRAHEDRON
    means: np.ndarray
    quats: np.ndarray
    dists: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.kind, self.means[idx].copy(), self.quats[idx].copy(),
                     self.dists[idx].copy(), self.opacity[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return self.subset(slice(None))


def focal_for_vfov(height: int, vfov_deg: float = 60.0) -> float:
    """Focal length in pixels for a vertical field of view."""
    return (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)


def make_camera(world_to_cam: np.ndarray, width: int, height: int,
                vfov_deg: float = 60.0) -> Camera:
    f = focal_for_vfov(height, vfov_deg)
    return Camera(np.asarray(world_to_cam, dtype=np.float32), np.float32(f),
                  np.float32(f), np.float32(width / 2.0), np.float32(height / 2.0),
                  int(width), int(height))


def look_at(position, target, width: int, height: int, up=(0.0, 1.0, 0.0),
            vfov_deg: float = 60.0) -> Camera:
    """Camera at ``position`` looking at ``target``; image y is world ``-up``."""
    p = np.asarray(position, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - p
    z /= np.linalg.norm(z)
    y0 = -np.asarray(up, dtype=np.float64)
    x = np.cross(y0, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    rot = np.stack([x, y, z])
    w2c = np.concatenate([rot, (-rot @ p)[:, None]], axis=1)
    return make_camera(w2c, width, height, vfov_deg)


def _random_rotations(rng, k: int) -> np.ndarray:
    """k random rotation matrices from the QR factorisation of Gaussian matrices."""
    out = np.empty((k, 3, 3))
    for i in range(k):
        a = rng.normal(size=(3, 3))
        q, r = np.linalg.qr(a)
        q = q * np.sign(np.diag(r))[None, :]
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out[i] = q
    return out


def gaussian_mixture(rng, n: int, k: int, extent: float) -> np.ndarray:
    """Room-scale point cloud: k flattened ("surface-like") Gaussian blobs.

    Component means are uniform in the cube [-extent/2, extent/2]^3, each has a
    random orientation and axis standard deviations (s, s, 0.05 s) with
    s ~ U(0.02, 0.1) * extent; weights are uniform and samples are clamped to
    the cube.
    """
    half = extent / 2.0
    centers = rng.uniform(-half, half, size=(k, 3))
    rots = _random_rotations(rng, k)
    scales = rng.uniform(0.02, 0.1, size=k) * extent
    comp = rng.integers(0, k, size=n)
    local = rng.normal(size=(n, 3))
    local *= np.stack([scales, scales, 0.05 * scales], axis=1)[comp]
    pts = np.einsum("nij,nj->ni", rots[comp], local) + centers[comp]
    return np.clip(pts, -half, half)


def _unit_quats(rng, n: int) -> np.ndarray:
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _finish(kind, means, quats, dists, opacity, sh, deg=3) -> Scene:
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(kind, f32(means), f32(quats), f32(dists), f32(opacity), f32(sh), deg)


def uniform_octahedra(n: int, seed: int = 0, box: float = 1.0,
                      dmin: float = 0.02, dmax: float = 0.1,
                      opacity_std: float = 1.0) -> Scene:
    """Centres U[-box, box]^3, log-uniform half-axes, N(0,0.2) degree-3 SH."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, size=(n, 3))
    quats = _unit_quats(rng, n)
    dists = np.exp(rng.uniform(math.log(dmin), math.log(dmax), size=(n, 3)))
    opacity = _sigmoid(rng.normal(0.0, opacity_std, size=n))
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    return _finish(OCTAHEDRON, means, quats, dists, opacity, sh)


def uniform_tetrahedra(n: int, seed: int = 0, box: float = 1.0,
                       dmin: float = 0.02, dmax: float = 0.1,
                       regular: bool = False) -> Scene:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, size=(n, 3))
    quats = _unit_quats(rng, n)
    if regular:
        s = np.exp(rng.uniform(math.log(dmin), math.log(dmax), size=n))
        dists = np.repeat(s[:, None], 4, axis=1)
    else:
        dists = np.exp(rng.uniform(math.log(dmin), math.log(dmax), size=(n, 4)))
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    return _finish(TETRAHEDRON, means, quats, dists, opacity, sh)


# --------------------------------------------------------------------------
# The measured workloads.
# --------------------------------------------------------------------------

def config0(seed: int = 0):
    """1,024 octahedra in [-1,1]^3 seen from distance 4 at 128x128."""
    scene = uniform_octahedra(1024, seed)
    w2c = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 4]], dtype=np.float32)
    cam = make_camera(w2c, 128, 128)
    return scene, [cam]


def config1(seed: int = 0):
    """100,000 regular tetrahedra from a 32-component mixture in [-5,5]^3, 1280x720."""
    rng = np.random.default_rng(seed)
    means = gaussian_mixture(rng, 100_000, 32, 10.0)
    quats = _unit_quats(rng, 100_000)
    s = np.exp(rng.uniform(math.log(0.005), math.log(0.05), size=100_000))
    dists = np.repeat(s[:, None], 4, axis=1)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=100_000))
    sh = rng.normal(0.0, 0.2, size=(100_000, 16, 3))
    scene = _finish(TETRAHEDRON, means, quats, dists, opacity, sh)
    cam = look_at((0.0, 0.0, -15.0), (0.0, 0.0, 0.0), 1280, 720)
    return scene, [cam]


def room_octahedra(n: int, seed: int = 0, extent: float = 20.0, k: int = 256) -> Scene:
    """Room-scale octahedra: mixture centres, log-normal(ln 0.02, 0.7) half-axes,
    opacity sigmoid(N(0, 1.5)), degree-3 SH ~ N(0, 0.2)."""
    rng = np.random.default_rng(seed)
    means = gaussian_mixture(rng, n, k, extent)
    quats = _unit_quats(rng, n)
    dists = np.exp(rng.normal(math.log(0.02), 0.7, size=(n, 3)))
    opacity = _sigmoid(rng.normal(0.0, 1.5, size=n))
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    return _finish(OCTAHEDRON, means, quats, dists, opacity, sh)


def circle_cameras(n_views: int, radius: float, sizes, seed: Optional[int] = None):
    """Cameras on a circle in the xz plane looking at the origin.

    ``sizes`` is either one (W, H) for every view or a list to draw from with
    ``default_rng(seed)``.
    """
    if isinstance(sizes, tuple):
        chosen = [sizes] * n_views
    else:
        rng = np.random.default_rng(seed)
        chosen = [sizes[i] for i in rng.integers(0, len(sizes), size=n_views)]
    cams = []
    for k in range(n_views):
        a = 2.0 * math.pi * k / n_views
        pos = (radius * math.cos(a), 0.0, radius * math.sin(a))
        cams.append(look_at(pos, (0.0, 0.0, 0.0), chosen[k][0], chosen[k][1]))
    return cams


def config2(seed: int = 0):
    """1,000,000 room-scale octahedra, one 1920x1080 camera at (8,0,0)."""
    scene = room_octahedra(1_000_000, seed)
    return scene, circle_cameras(16, 8.0, (1920, 1080))[:1]


MULTI_VIEW_SIZES = [(640, 480), (1280, 720), (1600, 1200), (1920, 1080)]


def config3(seed: int = 0):
    """500,000 room-scale octahedra, 16 views of mixed resolution."""
    scene = room_octahedra(500_000, seed)
    return scene, circle_cameras(16, 8.0, MULTI_VIEW_SIZES, seed=3)


def config4(seed: int = 0):
    """3,000,000 room-scale octahedra at extent 40 (step-loop workload)."""
    return room_octahedra(3_000_000, seed, extent=40.0)


def random_views(step: int, n_views: int = 8, radius: float = 16.0,
                 size=(1920, 1080), seed: int = 7) -> List[Camera]:
    rng = np.random.default_rng([seed, step])
    cams = []
    for _ in range(n_views):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        target = rng.normal(0.0, 1.0, size=3)
        up = (0.0, 1.0, 0.0) if abs(d[1]) < 0.95 else (1.0, 0.0, 0.0)
        cams.append(look_at(radius * d, target, size[0], size[1], up=up))
    return cams


def image_gradient(cams: List[Camera], seed: int = 1) -> np.ndarray:
    """dL/dC ~ N(0,1), all views packed view-major, each [3,H,W]."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=sum(3 * c.width * c.height for c in cams)).astype(np.float32)


def sparse_image_gradient(cams: List[Camera], frac: float, seed: int = 1) -> np.ndarray:
    """dL/dC ~ N(0,1) on a random fraction of pixels (all channels), zero elsewhere."""
    rng = np.random.default_rng(seed)
    parts = []
    for c in cams:
        hw = c.width * c.height
        g = rng.normal(size=(3, hw)).astype(np.float32)
        keep = rng.random(hw) < frac
        g[:, ~keep] = 0.0
        parts.append(g.reshape(-1))
    return np.concatenate(parts)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3}
