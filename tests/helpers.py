"""Small scene builders and independent reference formulas for the tests.

Nothing here calls the oracle's or the library's arithmetic: the formulas are
textbook results (Gaussian integrals, pinhole geometry) or library routines
(scipy rotations and spherical harmonics) used to pin the oracle.
"""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from paper_2412_03378_amd import scenes

SQRT2PI = math.sqrt(2.0 * math.pi)


def scene(means, scales, dens, quats=None, rgb=None, sh=None, deg=0):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    scales = np.broadcast_to(np.asarray(scales, np.float64), (n, 3)).copy()
    dens = np.broadcast_to(np.asarray(dens, np.float64), (n,)).copy()
    if quats is None:
        quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    if sh is None:
        rgb = np.ones((n, 3)) if rgb is None else np.broadcast_to(np.asarray(rgb, np.float64), (n, 3))
        sh = np.zeros((n, (deg + 1) ** 2, 3))
        sh[:, 0, :] = (rgb - 0.5) / scenes.Y00
    return scenes.Scene(np.float32(means), np.float32(quats), np.float32(scales),
                        np.float32(dens), np.float32(sh), deg)


def odd_camera(size=65, fov=40.0, distance=0.0):
    """Axis-aligned camera at (0,0,-distance); odd size so that the centre
    pixel's ray is the optical axis."""
    return scenes.axis_camera(distance, size, size, fov)


def rotation_matrix(q_wxyz):
    """Rotation of a (w,x,y,z) quaternion via scipy (scalar-last API)."""
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def pixel_ray_world(cam, px, py):
    """World origin and unit direction through pixel centre (px+0.5, py+0.5)."""
    Ri = np.linalg.inv(np.asarray(cam.R, np.float64))
    t = np.asarray(cam.t, np.float64)
    u = np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
    d = Ri @ u
    return -Ri @ t, d / np.linalg.norm(d)


def isotropic_x(kappa, s, r):
    """Line integral of kappa*exp(-|x-mu|^2/2s^2) along a line passing at
    distance r from mu: the 1D Gaussian integral s*sqrt(2 pi) times the
    peak exp(-r^2/2s^2)."""
    return kappa * SQRT2PI * s * math.exp(-r * r / (2 * s * s))


def point_line_distance(mu, o, d):
    v = np.asarray(mu, np.float64) - o
    return float(np.linalg.norm(v - np.dot(v, d) * d))


def real_sh_scipy(degree, v):
    """Real SH with Condon-Shortley phase built from scipy's complex SH:
    Y_l^m = sqrt2 Re Y_l^|m| (m>0), sqrt2 Im Y_l^|m| (m<0), Y_l^0."""
    from scipy.special import sph_harm_y
    v = np.asarray(v, np.float64)
    v = v / np.linalg.norm(v)
    polar = math.acos(max(-1.0, min(1.0, v[2])))
    azim = math.atan2(v[1], v[0])
    out = np.zeros((degree + 1) ** 2)
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            y = complex(sph_harm_y(l, abs(m), polar, azim))
            if m > 0:
                val = math.sqrt(2) * y.real
            elif m < 0:
                val = math.sqrt(2) * y.imag
            else:
                val = y.real
            out[l * l + l + m] = val
    return out
