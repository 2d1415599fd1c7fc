"""The X-ray cut (Sec. 6.2: I = sum of the line integrals x_i, terms below
x_min dropped) against the untruncated sum the oracle also reports: the sum
of every Gaussian's line integral on the ray, by brute force on a small
scene, and the bias of the cut on the X-ray workload at its x_min."""
import numpy as np

import oracle
import helpers as H
from paper_2412_03378_amd import scenes


def test_untruncated_sum_is_every_line_integral():
    """untrunc = sum of ray_integral's x over all Gaussians (brute force), and
    I = the same sum over the terms at or above x_min."""
    rng = np.random.default_rng(61)
    n = 40
    sc = H.scene(rng.uniform(-0.6, 0.6, (n, 3)), np.exp(rng.uniform(np.log(0.02), np.log(0.3), (n, 3))),
                 np.exp(rng.uniform(np.log(0.5), np.log(20), n)), quats=rng.standard_normal((n, 4)))
    cam = scenes.look_at([0.3, -0.2, -3.0], (0, 0, 0), 11, 9, 45.0)
    x_min = 1e-3
    r = oracle.render(sc, cam, oracle.Settings(mode="xray", x_min_xray=x_min))
    for py in range(0, cam.height, 2):
        for px in range(0, cam.width, 2):
            o, d = H.pixel_ray_world(cam, px, py)
            xs = np.array([oracle.ray_integral(sc.means[i], sc.quats[i], sc.scales[i], sc.dens[i],
                                               o, d)["x"] for i in range(n)])
            assert abs(r["untrunc"][py, px] - xs.sum()) <= 1e-12 * max(1.0, xs.sum())
            assert abs(r["image"][0, py, px] - xs[xs >= x_min].sum()) <= 1e-12 * max(1.0, xs.sum())


def _bias(x_min, views=(0, 21), n_pix=16):
    wl = scenes.config4(with_grad=False)
    worst = 0.0
    for v in views:
        cam = wl.cams[v]
        rng = np.random.default_rng(70 + v)
        pix = np.array([(cam.width // 2, cam.height // 2)]
                       + list(zip(rng.integers(0, cam.width, n_pix).tolist(),
                                  rng.integers(0, cam.height, n_pix).tolist())), np.int32)
        r = oracle.render(wl.scene, cam, oracle.Settings(mode="xray", x_min_xray=x_min), pixels=pix)
        worst = max(worst, float(((r["untrunc"] - r["image"][0]) / np.maximum(1.0, r["untrunc"])).max()))
    return worst


def test_xray_workload_truncation_bias():
    """At the X-ray workload's x_min the cut changes I by at most 1e-5 of
    max(1, I) on sampled pixels of two views; at 1e-6 it would not (which is
    why the workload uses the lower cut)."""
    b = _bias(scenes.XRAY_X_MIN)
    print(f"truncation bias at x_min {scenes.XRAY_X_MIN:g}: {b:.3g}")
    assert 0.0 <= b <= 1e-5
    assert _bias(1e-6) > 1e-5
