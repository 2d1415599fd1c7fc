"""CPU checks of the two screen-space bounds the rasteriser relies on, written
from their derivations (not from the kernel code):

1. The exact alpha bound: beta <= s_max gives x <= kappa sqrt(2 pi) s_max
   exp(-D^2/2), so alpha >= alpha_min needs D^2 <= D2max.  The pixels whose
   ray meets the ellipsoid {(x-m)^T Sigma^-1 (x-m) <= D2max} lie inside the
   bounding box of the conic with dual K (D2max Sigma - m m^T) K^T.  Every
   pixel where the oracle finds x >= tau must be inside that box.
2. The pre-test form f(d) = d^T Q d + 2 l^T d - 1 built from the record
   (a = A d, w = v0 + a) has the sign of D^2 - D'.
"""
import math

import numpy as np
import pytest

import oracle
import helpers as H
from paper_2412_03378_amd import scenes


def _view(cam, mu, q, s):
    R = cam.R.astype(np.float64)
    m = R @ np.asarray(mu, np.float64) + cam.t.astype(np.float64)
    Rc = R @ H.rotation_matrix(q)
    return m, Rc, np.asarray(s, np.float64)


def _bbox(cam, m, Rc, s, D2):
    K = np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1.0]])
    Sigma = Rc @ np.diag(s * s) @ Rc.T
    Cs = K @ (D2 * Sigma - np.outer(m, m)) @ K.T
    if Cs[2, 2] >= 0:
        return None
    out = []
    for a in (0, 1):
        disc = Cs[a, 2] ** 2 - Cs[a, a] * Cs[2, 2]
        r = np.sqrt(max(disc, 0.0))
        out += sorted([(Cs[a, 2] + r) / Cs[2, 2], (Cs[a, 2] - r) / Cs[2, 2]])
    return out  # x0, x1, y0, y1 in pixel coordinates (pixel centres at p + 0.5)


@pytest.mark.parametrize("seed,kernel", [(k, "gaussian") for k in range(4)] +
                         [(k, "epanechnikov") for k in range(4)])
def test_dual_conic_box_contains_every_visible_pixel(seed, kernel):
    """Gaussian: x <= kappa sqrt(2 pi) s_max exp(-D^2/2); Epanechnikov (Sec. 8,
    compact primitives): x <= (4/3) kappa s_max (1 - D^2)^(3/2), so x >= tau
    needs D^2 <= 1 - (tau / ((4/3) kappa s_max))^(2/3)."""
    rng = np.random.default_rng(seed)
    cam = scenes.look_at(rng.normal(0, 1, 3) * 0 + [0.3, -0.2, -3.0], (0, 0, 0), 64, 48, 45.0)
    tau = -math.log1p(-1.0 / 255.0)
    for _ in range(25):
        mu = np.float32(rng.uniform(-0.4, 0.4, 3))
        q = np.float32(rng.standard_normal(4))
        s = np.float32(np.exp(rng.uniform(np.log(0.01), np.log(0.12), 3)))
        kappa = float(np.float32(np.exp(rng.uniform(np.log(0.5), np.log(40)))))
        m, Rc, s64 = _view(cam, mu, q, s)
        epan = kernel == "epanechnikov"
        Kk = kappa * (4.0 / 3.0 if epan else math.sqrt(2 * math.pi)) * s64.max()
        if Kk <= tau:
            continue
        D2 = 1 - (tau / Kk) ** (2 / 3) if epan else 2 * math.log(Kk / tau)
        box = _bbox(cam, m, Rc, s64, D2)
        sc = H.scene([mu], [s], kappa, quats=[q])
        x = -np.log(oracle.render(sc, cam, oracle.Settings.no_thresholds(kernel=kernel))["T"])
        ys, xs = np.nonzero(x >= tau)
        if box is None or not len(xs):
            continue
        assert np.all(xs + 0.5 >= box[0] - 1e-6) and np.all(xs + 0.5 <= box[1] + 1e-6)
        assert np.all(ys + 0.5 >= box[2] - 1e-6) and np.all(ys + 0.5 <= box[3] + 1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_pre_test_form_has_the_sign_of_the_distance_excess(seed):
    rng = np.random.default_rng(100 + seed)
    cam = scenes.axis_camera(4.0, 96, 72, 50.0)
    for _ in range(40):
        mu = rng.uniform(-0.5, 0.5, 3)
        m, Rc, s = _view(cam, mu, rng.standard_normal(4), np.exp(rng.uniform(-4.5, -2, 3)))
        L = (Rc / s[None, :]).T
        A = L[:, :2] @ np.diag([1 / cam.fx, 1 / cam.fy])
        v0 = L @ (m / m[2])
        Dp = rng.uniform(2.0, 20.0)
        G = A.T @ A
        gv = A.T @ v0
        V = v0 @ v0
        Q = (m[2] ** 2 * (V * G - np.outer(gv, gv)) - Dp * G) / (Dp * V)
        l = -gv / V
        centre = np.array([cam.fx * m[0] / m[2] + cam.cx, cam.fy * m[1] / m[2] + cam.cy])
        for d in rng.normal(0, 25, (50, 2)):
            p = centre + d
            u = np.array([(p[0] - cam.cx) / cam.fx, (p[1] - cam.cy) / cam.fy, 1.0])
            w = L @ u
            pm = L @ m
            D2 = np.sum(np.cross(pm, w) ** 2) / (w @ w)      # Lagrange identity
            f = d @ Q @ d + 2 * l @ d - 1
            a = A @ d
            assert np.allclose(w, v0 + a)
            assert f == pytest.approx((w @ w) * (D2 - Dp) / (Dp * V), rel=1e-9, abs=1e-9)


def _row_interval(Q, l, c, ya, yb):
    """x-extent of {d : d^T Q d + 2 l^T d - 1 <= c} within the strip ya <= y <= yb,
    from the closed form the tile culling uses: centre d0 = -Q^-1 l,
    rho = 1 + c + l^T Q^-1 l, X = a Y -/+ sqrt(P - R Y^2), extreme X at the
    clamped Y of the leftmost / rightmost points (None if the strip misses)."""
    det = Q[0, 0] * Q[1, 1] - Q[0, 1] ** 2
    d0 = -np.linalg.solve(Q, l)
    rho = 1 + c - l @ d0
    a, P, R = -Q[0, 1] / Q[0, 0], rho / Q[0, 0], det / Q[0, 0] ** 2
    ymax = math.sqrt(rho * Q[0, 0] / det)
    yl = Q[0, 1] * math.sqrt(rho / (det * Q[1, 1]))
    lo, hi = max(ya - d0[1], -ymax), min(yb - d0[1], ymax)
    if lo > hi:
        return None
    y1 = min(max(yl, lo), hi)
    y2 = min(max(-yl, lo), hi)
    left = a * y1 - math.sqrt(max(P - R * y1 * y1, 0.0))
    right = a * y2 + math.sqrt(max(P - R * y2 * y2, 0.0))
    return d0[0] + left, d0[0] + right


@pytest.mark.parametrize("seed", range(4))
def test_culling_row_interval_is_the_strip_extent(seed):
    """Brute force over a dense grid: every point of the ellipse inside the
    strip lies in the closed-form interval, and both ends are reached."""
    rng = np.random.default_rng(200 + seed)
    for _ in range(30):
        B = rng.normal(0, 1, (2, 2))
        Q = B @ B.T + 0.05 * np.eye(2)
        Q /= rng.uniform(4, 60) ** 2
        l = rng.normal(0, 0.05, 2)
        c = 0.1
        d0 = -np.linalg.solve(Q, l)
        rho = 1 + c - l @ d0
        ext = 1.2 * math.sqrt(rho / np.linalg.eigvalsh(Q)[0])   # grid covers the ellipse
        ya = d0[1] + rng.uniform(-1.2, 1.0) * ext
        yb = ya + rng.uniform(0.5, 12.0)
        xs = np.linspace(d0[0] - ext, d0[0] + ext, 1201)
        ys = np.linspace(ya, yb, 61)
        X, Y = np.meshgrid(xs, ys)
        f = Q[0, 0] * X * X + 2 * Q[0, 1] * X * Y + Q[1, 1] * Y * Y + 2 * (l[0] * X + l[1] * Y) - 1
        inside = f <= c
        iv = _row_interval(Q, l, c, ya, yb)
        if iv is None:
            assert not inside.any()
            continue
        if not inside.any():
            continue
        step = xs[1] - xs[0]
        assert X[inside].min() >= iv[0] - 1e-9 and X[inside].max() <= iv[1] + 1e-9
        assert X[inside].min() <= iv[0] + 2 * step + 0.05 * ext / 60
        assert X[inside].max() >= iv[1] - 2 * step - 0.05 * ext / 60


def _beta_bound(cam, m, Rc, s, box):
    """Upper bound of beta = 1/|L u| over the rays of the pixel box, written
    from the derivation: |L u| >= |L u_c| - |u - u_c| / s_min, with the chord
    |u - u_c| largest at a corner of the box."""
    L = (Rc / s[None, :]).T
    uc = m / np.linalg.norm(m)
    chord = 0.0
    for X in (box[0], box[1]):
        for Y in (box[2], box[3]):
            u = np.array([(X - cam.cx) / cam.fx, (Y - cam.cy) / cam.fy, 1.0])
            chord = max(chord, np.linalg.norm(u / np.linalg.norm(u) - uc))
    den = np.linalg.norm(L @ uc) - chord / s.min()
    return s.max() if den <= 0 else min(s.max(), 1.0 / den)


@pytest.mark.parametrize("seed", range(4))
def test_beta_bound_contains_every_visible_pixel(seed):
    """The tighter bound D2max = 2 ln(kappa sqrt(2 pi) beta_bound / tau) still
    contains every pixel where the oracle finds x >= tau, beta_bound is never
    above s_max, and it is strictly below it for a Gaussian seen along its
    short axis."""
    rng = np.random.default_rng(300 + seed)
    cam = scenes.look_at([0.2, -0.3, -3.0], (0, 0, 0), 64, 48, 45.0)
    tau = -math.log1p(-1.0 / 255.0)
    tighter = 0
    for _ in range(25):
        mu = np.float32(rng.uniform(-0.4, 0.4, 3))
        q = np.float32(rng.standard_normal(4))
        s = np.float32(np.exp(rng.uniform(np.log(0.01), np.log(0.12), 3)))
        kappa = float(np.float32(np.exp(rng.uniform(np.log(0.5), np.log(40)))))
        m, Rc, s64 = _view(cam, mu, q, s)
        Kk = kappa * math.sqrt(2 * math.pi)
        if Kk * s64.max() <= tau:
            continue
        box = _bbox(cam, m, Rc, s64, 2 * math.log(Kk * s64.max() / tau))
        if box is None:
            continue
        beta = _beta_bound(cam, m, Rc, s64, box)
        assert beta <= s64.max() * (1 + 1e-12)
        tighter += beta < 0.9 * s64.max()
        sc = H.scene([mu], [s], kappa, quats=[q])
        x = -np.log(oracle.render(sc, cam, oracle.Settings.no_thresholds())["T"])
        ys, xs = np.nonzero(x >= tau)
        if not len(xs):
            continue
        L = (Rc / s64[None, :]).T
        pm = L @ m
        for px, py in zip(xs, ys):
            u = np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
            w = L @ u
            D2 = np.sum(np.cross(pm, w) ** 2) / (w @ w)
            assert Kk * beta > tau
            assert D2 <= 2 * math.log(Kk * beta / tau) + 1e-9
    assert tighter > 0
