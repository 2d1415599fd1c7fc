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
GRAD_REL = 1e-3         # |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 A_row) + ERR_K u E_row
ERR_K = 32


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


def _row_max(A):
    A = np.asarray(A, np.float64)
    if A.ndim >= 2:
        A = np.maximum(A, A.max(axis=-1, keepdims=True))
    return A


def grad_tolerance(ref, absref, errref=None):
    """Per-element bound GRAD_REL max(|g_ref|, 1e-2 A_row) + ERR_K u E_row.

    A_row is the largest sum of absolute per-pixel contributions over the
    components of the same Gaussian's parameter vector (mean, quaternion,
    scales, one SH coefficient's RGB): the FP32 arithmetic rotates these
    vectors, so each component's rounding error scales with the whole row.
    E_row (the oracle's err_* sums, row max likewise) is the FP32 error model:
    each pair's contribution without the cancellation of its upstream factor,
    weighted by how much a relative rounding error is amplified on its way
    (1 + D^2/2 through the exponential, one rounding per compositing step of
    the reverse replay); u = 2^-24 and ERR_K counts the roundings of one
    pair's chain (about 30 operations) with a small margin."""
    ref = np.asarray(ref, np.float64)
    tol = GRAD_REL * np.maximum(np.abs(ref), 1e-2 * _row_max(absref))
    if errref is not None:
        tol = tol + ERR_K * 2.0 ** -24 * _row_max(errref)
    return tol + 1e-30


def grad_errors(g, ref, absref, errref=None):
    """Worst ratio |g - g_ref| / grad_tolerance(...); <= 1 passes."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    r = np.abs(g - ref) / grad_tolerance(ref, absref, errref)
    return float(r.max()) if r.size else 0.0


def grad_worst(g, ref, absref, errref=None):
    """Description of the worst element (for test output)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    if not g.size:
        return "empty"
    r = np.abs(g - ref) / grad_tolerance(ref, absref, errref)
    k = np.unravel_index(int(np.argmax(r)), r.shape)
    A = _row_max(absref)[k]
    E = _row_max(errref)[k] if errref is not None else float("nan")
    return (f"at {tuple(int(x) for x in k)}: got {g[k]:.6g} ref {ref[k]:.6g} "
            f"|d|/A_row {abs(g[k] - ref[k]) / max(A, 1e-300):.3g} "
            f"|d|/(u E_row) {abs(g[k] - ref[k]) / max(2.0 ** -24 * E, 1e-300):.3g} ratio {r[k]:.3g}")
