"""Helpers for the GPU tests: move seeded scenes to the device, compare
against the oracle with the decision-margin rule.

A pixel whose oracle decisions (skip, clamp, stop) lie within MARGIN
(relative) of a threshold has two correct values up to rounding; such pixels
are compared with the loose FLIP_TOL (the size of one flipped decision) and
counted, all others with IMG_TOL.
"""
import numpy as np

IMG_TOL = 1e-4          # colour, absolute, per pixel and channel
XRAY_REL = 1e-4         # X-ray: |d| <= 1e-4 max(1, I_ref)
MARGIN = 1e-3           # relative decision margin that flags a pixel
FLIP_TOL = 0.05         # bound on the effect of one flipped decision
GRAD_REL = 1e-3         # |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 A_ref)


def device_scene(sc, dev):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    sh = t(sc.sh) if sc.sh is not None else None
    return t(sc.means), t(sc.quats), t(sc.scales), t(sc.dens), sh


def compare_image(img, ref, margin, xray=False):
    """img, ref: (C, P) or (C, H, W); margin: matching spatial shape.
    Returns (max error over unflagged pixels, n flagged, max error flagged)."""
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    ok = np.asarray(margin) > MARGIN
    if xray:
        err = np.abs(img - ref) / np.maximum(1.0, np.abs(ref))
    else:
        err = np.abs(img - ref)
    err = err.max(axis=0)
    e_ok = float(err[ok].max()) if ok.any() else 0.0
    e_flag = float(err[~ok].max()) if (~ok).any() else 0.0
    return e_ok, int((~ok).sum()), e_flag


def grad_errors(g, ref, absref):
    """Worst ratio |g - g_ref| / (GRAD_REL max(|g_ref|, 1e-2 A_row)); <= 1 passes.

    A_row is the largest sum of absolute per-pixel contributions over the
    components of the same Gaussian's parameter vector (mean, quaternion,
    scales, one SH coefficient's RGB): the FP32 arithmetic rotates these
    vectors, so each component's rounding error scales with the whole row."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    A = np.asarray(absref, np.float64)
    if A.ndim >= 2:
        A = np.maximum(A, A.max(axis=-1, keepdims=True))
    scale = GRAD_REL * np.maximum(np.abs(ref), 1e-2 * A) + 1e-30
    r = np.abs(g - ref) / scale
    return float(r.max()) if r.size else 0.0
