"""FP64 CPU oracle for volumetrically consistent Gaussian rasterisation.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the library never does.  It does not import the
library and the library does not import it.

The arithmetic lives in ``vgr_oracle.c`` (plain C, double precision, OpenMP
over pixels); this module only compiles it, marshals numpy arrays and
duck-typed scene / camera objects (attributes ``means, quats, scales, dens,
sh, sh_degree`` and ``R, t, fx, fy, cx, cy, width, height, znear``).

Passages followed (arXiv 2412.03378): the density mixture and Gaussian
(Sec. 3.2), the compact Epanechnikov primitive named as future work (Sec. 8), the 3DGS splatting opacity the paper compares against (Sec. 3,
eq. 3dgs_alpha, eq. affine_approx), the alpha-blend without splatting (Sec. 4.1), the 1D Gaussian on
a ray and its boxed full-line integral (Sec. 4.2, Supp. B), the density
reparameterisation (Sec. 5, eq. density_reparam), tomography as a sum of line
integrals (Sec. 6.2), and the world-space positional gradient norms that
drive densification (Supp. D).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vgr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_float),
                ("pad", C.c_int32)]


class _Settings(C.Structure):
    _fields_ = [("mode", C.c_int32), ("sh_degree", C.c_int32), ("act", C.c_int32),
                ("density", C.c_int32), ("alpha_model", C.c_int32), ("near_segment", C.c_int32),
                ("tile_resort", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("kernel", C.c_int32), ("pixel_window", C.c_int32), ("pad3", C.c_int32),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("T_min", C.c_double), ("x_min_xray", C.c_double), ("bg", C.c_double * 3),
                ("near_threshold", C.c_double)]


@dataclass
class Settings:
    """Thresholds of the compositing rule (defaults follow the 3DGS
    framework the paper builds on)."""
    mode: str = "color"            # "color" | "xray"
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    x_min_xray: float = 1e-6
    bg: tuple = (0.0, 0.0, 0.0)
    act: str = "clamp"             # "clamp" | "softplus"
    density: str = "kappa"         # "kappa" | "theta" (eq. density_reparam)
    alpha_model: str = "volumetric"  # "volumetric" | "splat" (3DGS, eq. 3dgs_alpha)
    near_segment: bool = False     # integrate each ray from the near plane on (Sec. 4.2)
    resort_tile: tuple = None      # (w, h): per-tile order by gamma on the tile-centre ray
    kernel: str = "gaussian"       # "gaussian" | "epanechnikov" (compact, Sec. 8)
    pixel_window: int = 0          # > 0 (with resort_tile): per-pixel re-sorting window

    @staticmethod
    def no_thresholds(mode="color", act="softplus", bg=(0.0, 0.0, 0.0), density="kappa",
                      near_segment=False, kernel="gaussian"):
        return Settings(mode=mode, alpha_min=1e-300, alpha_max=1.0 - 1e-12, T_min=0.0,
                        x_min_xray=1e-300, bg=bg, act=act, density=density,
                        near_segment=near_segment, kernel=kernel)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    fp = C.POINTER(C.c_float)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    lib.orc_ray_integral.argtypes = [fp, fp, fp, C.c_float, dp, dp, C.c_int, dp]
    lib.orc_sh_basis.argtypes = [C.c_int, dp, dp, dp]
    lib.orc_render.argtypes = [C.c_int64, fp, fp, fp, fp, fp, C.POINTER(_Cam),
                               C.POINTER(_Settings), C.c_int64, ip, dp, dp, lp, ip, dp, dp]
    lib.orc_render_backward.argtypes = [C.c_int64, fp, fp, fp, fp, fp, C.POINTER(_Cam),
                                        C.POINTER(_Settings), C.c_int64, ip, dp] + [dp] * 15
    lib.orc_max_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def _cam(cam) -> _Cam:
    c = _Cam()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32).reshape(3)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def _settings(st: Settings, sh_degree: int) -> _Settings:
    s = _Settings()
    s.mode = 1 if st.mode == "xray" else 0
    s.sh_degree = int(sh_degree)
    s.act = 1 if st.act == "softplus" else 0
    s.density = 1 if st.density == "theta" else 0
    s.alpha_model = 1 if st.alpha_model == "splat" else 0
    s.near_segment = 1 if st.near_segment else 0
    s.kernel = 1 if st.kernel == "epanechnikov" else 0
    if st.resort_tile:
        s.tile_resort = 1
        s.tile_w, s.tile_h = int(st.resort_tile[0]), int(st.resort_tile[1])
    s.pixel_window = int(st.pixel_window or 0)
    s.alpha_min, s.alpha_max = float(st.alpha_min), float(st.alpha_max)
    s.T_min, s.x_min_xray = float(st.T_min), float(st.x_min_xray)
    s.bg[:] = [float(v) for v in st.bg]
    return s


def all_pixels(cam) -> np.ndarray:
    ys, xs = np.mgrid[0:int(cam.height), 0:int(cam.width)]
    return np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32))


def _scene_arrays(scene, mode):
    means, quats = _f32(scene.means), _f32(scene.quats)
    scales, dens = _f32(scene.scales), _f32(scene.dens)
    sh = None
    if mode != "xray":
        sh = _f32(scene.sh)
    return means, quats, scales, dens, sh


def set_threads(n: int):
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def ray_integral(mean, quat, scale, dens, o, d, kernel="gaussian"):
    """Full-line integral of one Gaussian (or Epanechnikov primitive) along
    o + t d (d is normalised here).  Returns dict(gamma, beta, Gmax, x, alpha);
    Gmax = exp(-D^2/2) for either kernel."""
    lib = _load()
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    out = np.zeros(4, np.float64)
    lib.orc_ray_integral(_ptr(_f32(mean), C.c_float), _ptr(_f32(quat), C.c_float),
                         _ptr(_f32(scale), C.c_float), float(dens),
                         _ptr(np.ascontiguousarray(o, np.float64), C.c_double),
                         _ptr(np.ascontiguousarray(d), C.c_double),
                         1 if kernel == "epanechnikov" else 0, _ptr(out, C.c_double))
    g, b, G, x = out
    return dict(gamma=g, beta=b, Gmax=G, x=x, alpha=-math.expm1(-x))


def sh_basis(degree, v):
    """Real orthonormal SH (Condon-Shortley phase) at unit vector v:
    returns (Y[(deg+1)^2], dY[(deg+1)^2, 3]) (gradient of the polynomial
    extension)."""
    lib = _load()
    nb = (degree + 1) ** 2
    Y = np.zeros(nb, np.float64)
    dY = np.zeros((nb, 3), np.float64)
    rc = lib.orc_sh_basis(int(degree), _ptr(np.ascontiguousarray(v, np.float64), C.c_double),
                          _ptr(Y, C.c_double), _ptr(dY, C.c_double))
    if rc:
        raise ValueError("degree out of range")
    return Y, dY


def render(scene, cam, settings: Settings = None, pixels=None):
    """Render one view.  ``pixels``: (P, 2) int array of (x, y), or None for
    the whole image.  Returns dict with ``image`` ((C, P) or (C, H, W)),
    ``T`` (final transmittance), ``last`` (index of the last blended
    Gaussian, -1 if none), ``nblend``, the decision margins and ``untrunc``
    (X-ray sum without the x_min cut).

    Decision margins (vgr_oracle.c, dec_margin): ``margin_x`` is the smallest,
    over the tests of x or alpha against a threshold (skip, clamp, X-ray cut),
    of the relative distance to the threshold divided by the amplification of
    that value's FP32 rounding error (1 + D^2/2 for a line integral);
    ``margin_T`` the same for the termination tests T (1 - alpha) < T_min
    (amplification: the summed amplifications of the factors of T);
    ``margin_order`` (per-tile re-sorting only, else inf) the smallest
    relative gap between the order keys of two Gaussians that reach the
    pixel (per-tile keys, and with a pixel window the per-pixel gammas too).

    ``pixel_window`` W > 0 (with ``resort_tile``): the Gaussians that reach
    alpha_min at a pixel, in the per-tile order, pass through a window of W
    entries ordered by gamma on the pixel's own ray; the smallest leaves the
    window to be composited whenever it is full, the rest at the end.  W = 1
    is the per-tile order; W at least the number of such Gaussians is the
    exact per-pixel order by gamma."""
    lib = _load()
    st = settings or Settings()
    full = pixels is None
    pix = all_pixels(cam) if full else np.ascontiguousarray(np.asarray(pixels, np.int32))
    P = pix.shape[0]
    nch = 1 if st.mode == "xray" else 3
    means, quats, scales, dens, sh = _scene_arrays(scene, st.mode)
    out = np.zeros((P, nch), np.float64)
    T = np.zeros(P, np.float64)
    last = np.zeros(P, np.int64)
    nblend = np.zeros(P, np.int32)
    margin = np.zeros((P, 3), np.float64)
    untrunc = np.zeros(P, np.float64)
    cam_s, set_s = _cam(cam), _settings(st, scene.sh_degree)
    rc = lib.orc_render(int(means.shape[0]), _ptr(means, C.c_float), _ptr(quats, C.c_float),
                        _ptr(scales, C.c_float), _ptr(dens, C.c_float), _ptr(sh, C.c_float),
                        C.byref(cam_s), C.byref(set_s), P, _ptr(pix, C.c_int32),
                        _ptr(out, C.c_double), _ptr(T, C.c_double), _ptr(last, C.c_int64),
                        _ptr(nblend, C.c_int32), _ptr(margin, C.c_double),
                        _ptr(untrunc, C.c_double))
    if rc:
        raise RuntimeError(f"orc_render failed ({rc})")
    res = dict(image=out.T.copy(), T=T, last=last, nblend=nblend,
               margin_x=margin[:, 0].copy(), margin_T=margin[:, 1].copy(),
               margin_order=margin[:, 2].copy(), untrunc=untrunc, pixels=pix)
    if full:
        H, W = int(cam.height), int(cam.width)
        res["image"] = res["image"].reshape(nch, H, W)
        for k in ("T", "last", "nblend", "margin_x", "margin_T", "margin_order", "untrunc"):
            res[k] = res[k].reshape(H, W)
    return res


def render_backward(scene, cam, settings: Settings, dL, pixels=None, with_abs=True,
                    near_threshold=0.0):
    """Gradients of sum(dL * image) w.r.t. means, quats, scales, dens, sh for
    one view.  ``dL`` is (C, P) for a pixel list or (C, H, W) for the whole
    image.  Returns dict of FP64 gradients and, if ``with_abs``, the sums of
    absolute per-pixel contributions (``abs_*``) and the FP32 error scales
    (``err_*``: the same sums without cancellation of the upstream factor,
    each pair weighted by its rounding amplification) used for tolerances.

    ``near_threshold`` > 0 (X-ray mode only): chain only the pairs whose cut
    decision has a margin (as ``margin_x`` of render) below it, on either side
    of the cut; ``abs_*`` then bounds what flipping those decisions can change
    in each gradient element."""
    lib = _load()
    st = settings or Settings()
    if near_threshold > 0 and st.mode != "xray":
        raise ValueError("near_threshold applies to X-ray mode only")
    full = pixels is None
    pix = all_pixels(cam) if full else np.ascontiguousarray(np.asarray(pixels, np.int32))
    P = pix.shape[0]
    nch = 1 if st.mode == "xray" else 3
    g = np.ascontiguousarray(np.asarray(dL, np.float64).reshape(nch, P).T)
    means, quats, scales, dens, sh = _scene_arrays(scene, st.mode)
    n = means.shape[0]
    nb = (scene.sh_degree + 1) ** 2
    shapes = dict(means=(n, 3), quats=(n, 4), scales=(n, 3), dens=(n,), sh=(n, nb, 3))
    grads = {k: np.zeros(s, np.float64) for k, s in shapes.items()}
    absg = {k: (np.zeros(s, np.float64) if with_abs else None) for k, s in shapes.items()}
    errg = {k: (np.zeros(s, np.float64) if with_abs else None) for k, s in shapes.items()}
    cam_s, set_s = _cam(cam), _settings(st, scene.sh_degree)
    set_s.near_threshold = float(near_threshold)
    keys = ("means", "quats", "scales", "dens", "sh")
    rc = lib.orc_render_backward(
        int(n), _ptr(means, C.c_float), _ptr(quats, C.c_float), _ptr(scales, C.c_float),
        _ptr(dens, C.c_float), _ptr(sh, C.c_float), C.byref(cam_s), C.byref(set_s), P,
        _ptr(pix, C.c_int32), _ptr(g, C.c_double),
        *[_ptr(grads[k], C.c_double) for k in keys],
        *[_ptr(absg[k], C.c_double) for k in keys],
        *[_ptr(errg[k], C.c_double) for k in keys])
    if rc:
        raise RuntimeError(f"orc_render_backward failed ({rc})")
    res = dict(grads)
    if with_abs:
        for k in keys:
            res["abs_" + k] = absg[k]
            res["err_" + k] = errg[k]
    return res


def densify_stats(scene, cams, settings: Settings, dLs):
    """Densification statistics of one multi-view step (Supp. D: world-space
    positional gradients): per Gaussian, the sum over views of the norm of
    that view's dL/dmu, with the loss of view v being sum(dLs[v] * image_v).

    Which views count a Gaussian as visible depends on the tile bound of an
    implementation, so two bounds are returned: ``visible_lo`` counts the
    views where it contributes to some pixel (blended or summed), ``visible_hi``
    the views where it survives the near-plane and opacity culls
    (kappa sqrt(2 pi) s_max >= the skip threshold, the largest x any ray can
    reach, since beta <= s_max; for the splatting model, peak opacity >=
    alpha_min).  Also returned: the per-view gradients and
    their sums of absolute contributions and error scales, for tolerances."""
    st = settings or Settings()
    xray = st.mode == "xray"
    n = int(np.asarray(scene.means).shape[0])
    norm_sum = np.zeros(n)
    lo = np.zeros(n, np.int64)
    hi = np.zeros(n, np.int64)
    per_view = []
    s32 = _f32(scene.scales)
    dens = _f32(scene.dens)
    if st.density == "theta":
        th = np.clip(dens.astype(np.float64), 0.0, 1.0)
        kappa = -np.log1p(-0.99 * th) * (1.0 / s32.astype(np.float64)).sum(1) / 3.0
    else:
        kappa = dens.astype(np.float64)
    tau = st.x_min_xray if xray else -math.log1p(-st.alpha_min)
    reach = kappa * math.sqrt(2.0 * math.pi) * s32.max(1).astype(np.float64)
    if st.alpha_model == "splat":
        # splatting model: alpha <= o, so a Gaussian can reach alpha_min only
        # if its peak opacity does
        alive = np.clip(dens.astype(np.float64), 0.0, 1.0) >= st.alpha_min * (1.0 - 1e-6)
    else:
        alive = reach >= tau * (1.0 - 1e-5)
    means = _f32(scene.means)
    for cam, dL in zip(cams, dLs):
        r = render_backward(scene, cam, st, dL, with_abs=True)
        per_view.append(r)
        norm_sum += np.linalg.norm(r["means"], axis=1)
        touched = (r["abs_dens"] > 0) | (r["abs_means"].max(1) > 0)
        if not xray:
            touched |= r["abs_sh"].reshape(n, -1).max(1) > 0
        lo += touched
        # view-space depth of the mean in FP64; the FP32 depth key that decides
        # the near cull differs by rounding only, so the bound is relaxed by 1e-6
        R = np.asarray(cam.R, np.float32).reshape(3, 3).astype(np.float64)
        t = np.asarray(cam.t, np.float32).reshape(3).astype(np.float64)
        z = means.astype(np.float64) @ R[2] + t[2]
        znear = float(getattr(cam, "znear", 0.2))
        hi += (z > znear - 1e-6 * max(1.0, abs(znear))) & alive
    return dict(norm_sum=norm_sum, visible_lo=lo, visible_hi=hi, per_view=per_view)
