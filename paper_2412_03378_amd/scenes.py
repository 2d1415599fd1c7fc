"""Seeded synthetic inputs: cameras, Gaussian scenes and upstream gradients.

This module only draws random numbers and builds camera poses.  It holds none
of the renderer's arithmetic, so both the HIP path and the FP64 oracle can be
fed from it without sharing any code with each other.

The paper evaluates on Mip-NeRF360 / Tanks&Temples / DeepBlending scenes of
1.5M-5.3M Gaussians (Supp. E) and on the R2-Gaussian CT sets (Sec. 6.2); none
of those are available, so the workloads below are synthetic stand-ins with the
same sizes and structure.

Conventions
-----------
* Cameras use OpenCV axes (x right, y down, z forward).  ``R`` and ``t`` map a
  world point to view space: ``x_v = R x_w + t``.  Focal lengths come from the
  horizontal field of view, ``f = W / (2 tan(fov/2))``, principal point at the
  image centre, pixel centres at ``+0.5``.
* Quaternions are ``(w, x, y, z)``; scales are linear and positive; densities
  ``kappa`` are the mixture weights of the density field (Sec. 3.2), in
  1/length.
* SH coefficients are stored ``[n, (deg+1)^2, 3]``, basis index ``k = l^2+l+m``.
  A plain RGB colour ``rgb`` is stored as the DC coefficient
  ``(rgb - 0.5) / Y_00`` with ``Y_00 = 1/(2 sqrt(pi))`` so that the evaluated
  colour (DC term plus the 0.5 offset) equals ``rgb``.

Every generator draws from ``numpy.random.default_rng(seed)`` in the fixed
order cameras -> means -> scales -> quats -> density -> colour/SH.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

Y00 = 0.5 / math.sqrt(math.pi)


@dataclass
class Camera:
    """Pinhole camera; ``R`` row-major world->view rotation, ``t`` translation."""
    R: np.ndarray            # (3, 3) float32
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    def __post_init__(self):
        # the renderer receives FP32 camera parameters; keep the stored ones
        # exactly representable so that every consumer sees the same values
        self.R = np.ascontiguousarray(np.asarray(self.R, np.float32).reshape(3, 3))
        self.t = np.ascontiguousarray(np.asarray(self.t, np.float32).reshape(3))
        for k in ("fx", "fy", "cx", "cy", "znear"):
            setattr(self, k, float(np.float32(getattr(self, k))))
        self.width, self.height = int(self.width), int(self.height)

    @property
    def center(self) -> np.ndarray:
        """World-space camera centre ``-R^-1 t`` (float64; the stored FP32
        rotation is only approximately orthonormal)."""
        return -np.linalg.solve(self.R.astype(np.float64), self.t.astype(np.float64))


@dataclass
class Scene:
    means: np.ndarray        # (n, 3) float32
    quats: np.ndarray        # (n, 4) float32, (w, x, y, z), not normalised
    scales: np.ndarray       # (n, 3) float32, > 0
    dens: np.ndarray         # (n,) float32, >= 0
    sh: Optional[np.ndarray]  # (n, (deg+1)^2, 3) float32 or None (X-ray)
    sh_degree: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.quats[idx], self.scales[idx],
                     self.dens[idx], None if self.sh is None else self.sh[idx],
                     self.sh_degree)


@dataclass
class Workload:
    name: str
    scene: Scene
    cams: List[Camera]
    mode: str = "color"      # "color" | "xray"
    tile: tuple = (16, 16)
    bg: tuple = (0.0, 0.0, 0.0)
    dL: Optional[List[np.ndarray]] = None   # upstream gradients, one per view
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# camera construction

def focal_from_fov(width: int, fov_deg: float) -> float:
    return width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))


def look_at(eye, target, width, height, fov_deg, znear=0.2,
            down_hint=(0.0, 1.0, 0.0), alt_down_hint=(0.0, 0.0, 1.0),
            focal=None) -> Camera:
    """OpenCV look-at camera.  The image 'down' axis follows ``down_hint``
    (world +y, i.e. up = -y) unless the view direction is within ~8 deg of it,
    in which case ``alt_down_hint`` (world +z) is used."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    z = target - eye
    z /= np.linalg.norm(z)
    hint = np.asarray(down_hint, np.float64)
    if abs(float(np.dot(z, hint / np.linalg.norm(hint)))) > 0.99:
        hint = np.asarray(alt_down_hint, np.float64)
    x = np.cross(hint, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    f = focal_from_fov(width, fov_deg) if focal is None else float(focal)
    return Camera(R.astype(np.float32), t.astype(np.float32), f, f,
                  width / 2.0, height / 2.0, int(width), int(height), znear)


def axis_camera(distance, width, height, fov_deg, znear=0.2) -> Camera:
    """Camera at (0, 0, -distance) looking along +z at the origin (R = I)."""
    f = focal_from_fov(width, fov_deg)
    return Camera(np.eye(3, dtype=np.float32),
                  np.array([0.0, 0.0, distance], np.float32), f, f,
                  width / 2.0, height / 2.0, int(width), int(height), znear)


# ----------------------------------------------------------------------------
# random draws

def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _random_rotation(rng):
    a = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))[None, :]
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def clustered_means(rng, n, n_clusters, box=3.0, std_range=(0.05, 0.5)):
    """Mixture of anisotropic Gaussian clusters inside [-box, box]^3 (equal
    weights; samples falling outside the box are re-drawn)."""
    centres = rng.uniform(-box, box, (n_clusters, 3))
    stds = _log_uniform(rng, std_range[0], std_range[1], (n_clusters, 3))
    rots = np.stack([_random_rotation(rng) for _ in range(n_clusters)])
    assign = rng.integers(0, n_clusters, n)
    out = np.empty((n, 3), np.float64)
    todo = np.arange(n)
    while todo.size:
        c = assign[todo]
        local = rng.standard_normal((todo.size, 3)) * stds[c]
        pts = centres[c] + np.einsum("nij,nj->ni", rots[c], local)
        ok = np.all(np.abs(pts) <= box, axis=1)
        out[todo[ok]] = pts[ok]
        todo = todo[~ok]
    return out


def _sh_random(rng, n, degree, std):
    k = (degree + 1) ** 2
    out = rng.standard_normal((n, k, 3), dtype=np.float32)
    out *= np.float32(std)
    return out


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def _scene(means, scales, quats, dens, sh, deg):
    return Scene(_f32(means), _f32(quats), _f32(scales), _f32(dens),
                 None if sh is None else _f32(sh), deg)


# ----------------------------------------------------------------------------
# the five workloads

def config1(n=1000, width=128, height=128, seed=1) -> Workload:
    """128x128, fov 60, camera at (0,0,-4) looking at the origin; uniform
    means in [-1,1]^3, log-uniform scales [0.01, 0.1], random rotations,
    log-uniform density [0.1, 10], RGB uniform [0,1] as SH degree 0."""
    rng = np.random.default_rng(seed)
    cam = axis_camera(4.0, width, height, 60.0)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    scales = _log_uniform(rng, 0.01, 0.1, (n, 3))
    quats = _unit_quats(rng, n)
    dens = _log_uniform(rng, 0.1, 10.0, n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh = ((rgb - 0.5) / Y00)[:, None, :]
    return Workload("single view 128x128, 1k Gaussians, SH0",
                    _scene(means, scales, quats, dens, sh, 0), [cam])


def with_theta(scene: Scene, seed: int, lo: float = 0.02, hi: float = 0.98) -> Scene:
    """The same Gaussians with the density input replaced by the paper's
    density parameter theta (Sec. 5), drawn uniform in [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    theta = _f32(rng.uniform(lo, hi, scene.n))
    return Scene(scene.means, scene.quats, scene.scales, theta, scene.sh, scene.sh_degree)


def with_opacity(scene: Scene, seed: int, lo: float = 0.05, hi: float = 1.0) -> Scene:
    """The same Gaussians with the density input replaced by a peak opacity
    in [lo, hi] (seeded), the input of the 3DGS splatting model (Sec. 3)."""
    rng = np.random.default_rng(seed)
    o = _f32(rng.uniform(lo, hi, scene.n))
    return Scene(scene.means, scene.quats, scene.scales, o, scene.sh, scene.sh_degree)


def _clustered_scene(rng, n, n_clusters, sh_degree=3):
    means = clustered_means(rng, n, n_clusters)
    scales = np.exp(rng.normal(math.log(0.01), 0.7, (n, 3)))
    quats = _unit_quats(rng, n)
    dens = _log_uniform(rng, 0.1, 50.0, n)
    sh = _sh_random(rng, n, sh_degree, 0.2)
    return _scene(means, scales, quats, dens, sh, sh_degree)


def _upstream(rng, cams, channels=3):
    return [rng.standard_normal((channels, c.height, c.width), dtype=np.float32) for c in cams]


def config2(n=1_000_000, width=1920, height=1080, n_clusters=64, seed=2,
            with_grad=True) -> Workload:
    """1920x1080, fov 50, camera at (0,0,-8) looking at the origin; 1M
    Gaussians from 64 clusters, log-normal scales, density log-uniform
    [0.1, 50], SH degree 3 coefficients N(0, 0.2); dL/dimage ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    cam = axis_camera(8.0, width, height, 50.0)
    scene = _clustered_scene(rng, n, n_clusters)
    dL = _upstream(rng, [cam]) if with_grad else None
    return Workload(f"single view {width}x{height}, {n} Gaussians, SH3",
                    scene, [cam], dL=dL)


_RESOLUTIONS = [(640, 480), (1280, 720), (1600, 1064), (1920, 1080)]


def _sphere_dirs(rng, k):
    v = rng.standard_normal((k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def config3(n=3_000_000, n_views=16, n_clusters=256, seed=3,
            with_grad=True) -> Workload:
    """16 cameras on a sphere of radius 6 looking at the origin, resolutions
    drawn from {640x480, 1280x720, 1600x1064, 1920x1080}, fov 50; 3M
    clustered Gaussians (256 clusters), SH degree 3."""
    rng = np.random.default_rng(seed)
    dirs = _sphere_dirs(rng, n_views)
    res = rng.integers(0, len(_RESOLUTIONS), n_views)
    cams = [look_at(6.0 * d, (0, 0, 0), *_RESOLUTIONS[r], 50.0)
            for d, r in zip(dirs, res)]
    scene = _clustered_scene(rng, n, n_clusters)
    dL = _upstream(rng, cams) if with_grad else None
    return Workload(f"batched {n_views} views mixed resolution, {n} Gaussians, SH3",
                    scene, cams, dL=dL)


def xray_cameras(n_views=64, size=512, source_dist=4.0, det_dist=2.0,
                 det_side=3.2, znear=0.2):
    """Cone-beam geometry: source on a circle of radius ``source_dist`` about
    the world z axis, detector plane ``det_dist`` beyond the origin, square
    detector of side ``det_side`` sampled at ``size``^2 pixels."""
    f = (source_dist + det_dist) / (det_side / size)
    cams = []
    for k in range(n_views):
        a = 2.0 * math.pi * k / n_views
        eye = (source_dist * math.cos(a), source_dist * math.sin(a), 0.0)
        cams.append(look_at(eye, (0, 0, 0), size, size, 0.0, znear,
                            down_hint=(0.0, 0.0, -1.0),
                            alt_down_hint=(0.0, 1.0, 0.0), focal=f))
    return cams


# Cut x_min of the X-ray workload: dropping the terms below the cut biases the
# sum I = sum x_i low; at 1e-6 the bias reaches 2.8e-5 of max(1, I) on this
# scene, at 1e-7 it stays near 5e-6, below the 1e-5 the workload allows
# (checked on sampled pixels against the untruncated sum).
XRAY_X_MIN = 1e-7


def config4(n=500_000, n_views=64, size=512, seed=4, with_grad=True) -> Workload:
    """X-ray tomography: 500k Gaussians, means uniform in the unit ball,
    log-uniform scales [0.002, 0.05], density log-uniform [0.5, 20], no
    colour; 64 cone-beam projections 512x512."""
    rng = np.random.default_rng(seed)
    cams = xray_cameras(n_views, size)
    dirs = _sphere_dirs(rng, n)
    radius = rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    means = dirs * radius[:, None]
    scales = _log_uniform(rng, 0.002, 0.05, (n, 3))
    quats = _unit_quats(rng, n)
    dens = _log_uniform(rng, 0.5, 20.0, n)
    scene = _scene(means, scales, quats, dens, None, 0)
    dL = _upstream(rng, cams, channels=1) if with_grad else None
    return Workload(f"xray {n_views} cone-beam views {size}x{size}, {n} Gaussians",
                    scene, cams, mode="xray", dL=dL)


def config5(n=6_000_000, n_views=64, n_clusters=1024, width=1920, height=1080,
            seed=5, with_grad=True) -> Workload:
    """Training-step scale: 6M Gaussians (1024 clusters), SH degree 3, 64
    views at 1920x1080 on a sphere of radius U[5, 8] looking at the origin."""
    rng = np.random.default_rng(seed)
    dirs = _sphere_dirs(rng, n_views)
    radii = rng.uniform(5.0, 8.0, n_views)
    cams = [look_at(r * d, (0, 0, 0), width, height, 50.0)
            for d, r in zip(dirs, radii)]
    scene = _clustered_scene(rng, n, n_clusters)
    dL = _upstream(rng, cams) if with_grad else None
    return Workload(f"training step {n_views} views {width}x{height}, {n} Gaussians, SH3",
                    scene, cams, dL=dL)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
