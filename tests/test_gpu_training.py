"""GPU parity of the training-side options: the density reparameterisation
(Sec. 5, eq. density_reparam) computed inside the preprocess, and the
densification statistics (Supp. D: per-Gaussian world-space positional
gradient norms and visible-view counts) accumulated by the backward.
Everything goes through the C ABI and is compared with the FP64 oracle.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import gpu_helpers as G
import helpers as H
from paper_2412_03378_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def R(dev):
    from paper_2412_03378_amd import Renderer
    return Renderer(0)


def _settings(**kw):
    from paper_2412_03378_amd import Settings
    return Settings(**kw)


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, x_min_xray=st.x_min_xray, bg=st.bg, act=st.act,
                           density=st.density, alpha_model=st.alpha_model,
                           near_segment=st.near_segment)


KEYS = ("means", "quats", "scales", "dens", "sh")


def _multi_view_check(R, dev, sc, cams, st, seed):
    """Forward of all views in one call and the backward of the sum of the
    views' losses against the oracle; returns (grads, oracle stats)."""
    ost = _oset(st)
    xray = st.mode == "xray"
    t = G.device_scene(sc, dev)
    imgs = R.forward(*t, cams, st)
    rng = np.random.default_rng(seed)
    dLs = []
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, ost)
        img = imgs[v].cpu().numpy()
        G.check_image(img[None] if xray else img, ref, xray=xray, label=f"view {v}: ")
        dLs.append(G.upstream(rng, ref, 1 if xray else 3, xray))
    keys = KEYS[:4] if xray else KEYS
    grads = [torch.zeros_like(x) for x in t[:len(keys)]]
    dl_dev = [torch.from_numpy((d[0] if xray else d).astype(np.float32)).to(dev) for d in dLs]
    R.backward(dl_dev, *grads, *([None] if xray else []))
    torch.cuda.synchronize()
    ds = oracle.densify_stats(sc, cams, ost, dLs)
    ds["flips"] = ([oracle.render_backward(sc, cam, ost, d, near_threshold=G.MARGIN_X)
                    for cam, d in zip(cams, dLs)] if xray else None)
    G.check_grads({k: g.cpu().numpy() for k, g in zip(keys, grads)},
                  G.sum_backward(ds["per_view"], keys, ds["flips"]))
    return grads, ds, dl_dev, t


def _norm_tolerance(ds):
    """Per Gaussian: sum over views of the Euclidean norm of the per-element
    gradient tolerance of dL_v/dmu (|(|g| - |g_ref|)| <= |g - g_ref|)."""
    tol = 0.0
    flips = ds.get("flips") or [None] * len(ds["per_view"])
    for pv, fv in zip(ds["per_view"], flips):
        tv = G.grad_tolerance(pv["means"], pv["abs_means"], pv["err_means"],
                              None if fv is None else fv["abs_means"])
        tol = tol + np.linalg.norm(tv, axis=1)
    return tol


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_theta_colour_single_view(R, dev, tile):
    """128x128, 1000 Gaussians (the parity workload) with theta in
    [0.02, 0.98] as the density input: image, dL/dtheta and the scales'
    extra path through kappa."""
    wl = scenes.config1()
    sc = scenes.with_theta(wl.scene, seed=41)
    st = _settings(act="softplus", tile=tile, bg=(0.1, 0.2, 0.3), density="theta")
    _multi_view_check(R, dev, sc, wl.cams, st, seed=42)


def test_theta_xray_multi_view(R, dev):
    """X-ray mode, three cone-beam views of 96x96 in one call, theta input."""
    wl = scenes.config4(n=3000, n_views=64, size=96, seed=4, with_grad=False)
    sc = scenes.with_theta(wl.scene, seed=43)
    cams = [wl.cams[k] for k in (0, 16, 40)]
    st = _settings(mode="xray", tile=(8, 8), density="theta")
    _multi_view_check(R, dev, sc, cams, st, seed=44)


@pytest.mark.parametrize("density", ["kappa", "theta", "splat"])
def test_densify_stats_multi_view(R, dev, density):
    """Three views of uneven size in one call: the per-Gaussian sum of
    |dL_v/dmu| matches the oracle within the gradient tolerance, the view
    count lies between the oracle's bounds, and a second backward adds the
    same amounts again."""
    wl = scenes.config3(n=1500, n_views=3, n_clusters=24, seed=45, with_grad=False)
    sc = wl.scene
    if density == "theta":
        sc = scenes.with_theta(sc, seed=46)
    if density == "splat":   # the statistics of the splatting comparison model
        sc = scenes.with_opacity(sc, seed=46)
    cams = [scenes.Camera(c.R, c.t, c.fx / 16, c.fy / 16, c.cx / 16, c.cy / 16,
                          c.width // 16, c.height // 16) for c in wl.cams]
    if density == "splat":
        st = _settings(sh_degree=3, act="softplus", tile=(16, 8), alpha_model="splat")
    else:
        st = _settings(sh_degree=3, act="softplus", tile=(16, 8), density=density)
    n = sc.n
    gnorm = torch.zeros(n, dtype=torch.float32, device=dev)
    vcount = torch.zeros(n, dtype=torch.int32, device=dev)
    R.set_densify_stats(gnorm, vcount)
    try:
        grads, ds, dl_dev, t = _multi_view_check(R, dev, sc, cams, st, seed=47)
        g1 = gnorm.cpu().numpy().astype(np.float64)
        c1 = vcount.cpu().numpy()
        tol = _norm_tolerance(ds)
        err = np.abs(g1 - ds["norm_sum"]) / (tol + 1e-30)
        k = int(np.argmax(err))
        print(f"norm ratio {err.max():.3g} at {k}: {g1[k]:.6g} vs {ds['norm_sum'][k]:.6g}")
        assert err.max() <= 1.0
        lo, hi = ds["visible_lo"], ds["visible_hi"]
        print("visible: lo", lo.sum(), "gpu", c1.sum(), "hi", hi.sum())
        assert np.all(c1 >= lo) and np.all(c1 <= hi)
        assert lo.sum() > 0 and (hi > lo).any()
        # a second backward of the same forward adds the same amounts again
        # (up to the order of the rasteriser's FP32 atomics)
        R.backward(dl_dev, *[torch.zeros_like(x) for x in grads], accumulate=True)
        torch.cuda.synchronize()
        g2 = gnorm.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g2 - 2 * ds["norm_sum"]) <= 2 * tol + 1e-30)
        assert np.array_equal(vcount.cpu().numpy(), 2 * c1)
    finally:
        R.set_densify_stats(None, None)


def test_densify_stats_graph_replays_match_eager(dev):
    """A captured step with the statistics on adds what the eager steps add:
    after the capture's own eager step and three replays, the view counts
    equal those of four eager steps exactly and the norm sums up to the order
    of the rasteriser's FP32 atomics."""
    from paper_2412_03378_amd import Renderer
    wl = scenes.config1(n=800, width=64, height=48)
    sc = scenes.with_theta(wl.scene, seed=48)
    st = _settings(act="softplus", tile=(8, 8), density="theta")
    t = G.device_scene(sc, dev)
    cam = wl.cams[0]
    dL = [torch.from_numpy(np.random.default_rng(49).standard_normal(
        (3, cam.height, cam.width)).astype(np.float32)).to(dev)]
    n = sc.n
    res = []
    for graph in (False, True):
        r = Renderer(0)
        gnorm = torch.zeros(n, dtype=torch.float32, device=dev)
        vcount = torch.zeros(n, dtype=torch.int32, device=dev)
        r.set_densify_stats(gnorm, vcount)
        outs = [torch.empty((3, cam.height, cam.width), device=dev)]
        grads = [torch.zeros_like(x) for x in t]
        if graph:
            r.graph_capture(t, [cam], st, outs, dL, grads)
            for _ in range(3):
                r.graph_launch()
                torch.cuda.synchronize()
            r.graph_check()
        else:
            for _ in range(4):
                r.forward(*t, [cam], st, outs)
                r.backward(dL, *grads, accumulate=False)
                torch.cuda.synchronize()
        res.append((gnorm.cpu().numpy(), vcount.cpu().numpy()))
        r.close()
    a, b = res[0][0].astype(np.float64), res[1][0].astype(np.float64)
    assert np.all(np.abs(a - b) <= G.GRAD_REL * np.maximum(np.abs(a), 1e-2 * a.max()))
    assert np.array_equal(res[0][1], res[1][1])
    assert res[0][1].max() == 4 and a.max() > 0


def test_densify_capacity_and_bad_density(R, dev):
    """Arrays shorter than the scene make the backward fail cleanly; an
    unknown density setting is rejected by the forward."""
    from paper_2412_03378_amd import _lib as L
    from paper_2412_03378_amd.renderer import camera_struct
    wl = scenes.config1(n=200, width=32, height=32)
    t = G.device_scene(wl.scene, dev)
    cam = wl.cams[0]
    st = _settings(tile=(8, 8))
    R.forward(*t, [cam], st)
    short = torch.zeros(100, dtype=torch.float32, device=dev)
    R.set_densify_stats(short, None)
    try:
        with pytest.raises(L.VgrError) as ei:
            R.backward([torch.ones((3, 32, 32), device=dev)],
                       *[torch.zeros_like(x) for x in t])
        assert ei.value.code == L.VGR_ERR_INVALID_ARG
        assert float(short.abs().sum()) == 0.0
    finally:
        R.set_densify_stats(None, None)
    bad = st.to_c()
    bad.density = 7
    outs = (C.c_void_p * 1)(torch.empty((3, 32, 32), device=dev).data_ptr())
    cams = (L.vgr_camera * 1)(camera_struct(cam))
    ptr = lambda x: C.c_void_p(x.data_ptr())
    rc = R._lib.vgr_render_forward(R._h, C.byref(bad), wl.scene.n, *[ptr(x) for x in t], 1,
                                   cams, outs)
    assert rc == L.VGR_ERR_INVALID_ARG


def test_densify_stats_xray(R, dev):
    """X-ray mode over three cone-beam views (no colour term in dL/dmu)."""
    wl = scenes.config4(n=2000, n_views=64, size=64, seed=4, with_grad=False)
    sc = wl.scene
    cams = [wl.cams[k] for k in (0, 21, 43)]
    st = _settings(mode="xray", tile=(8, 8))
    n = sc.n
    gnorm = torch.zeros(n, dtype=torch.float32, device=dev)
    vcount = torch.zeros(n, dtype=torch.int32, device=dev)
    R.set_densify_stats(gnorm, vcount)
    try:
        _, ds, _, _ = _multi_view_check(R, dev, sc, cams, st, seed=66)
        g1 = gnorm.cpu().numpy().astype(np.float64)
        c1 = vcount.cpu().numpy()
        err = np.abs(g1 - ds["norm_sum"]) / (_norm_tolerance(ds) + 1e-30)
        print(f"norm ratio {err.max():.3g}")
        assert err.max() <= 1.0
        assert np.all(c1 >= ds["visible_lo"]) and np.all(c1 <= ds["visible_hi"])
    finally:
        R.set_densify_stats(None, None)


@pytest.mark.parametrize("opt", [{"density": "theta"}, {"alpha_model": "splat"},
                                 {"near_segment": True}, {"tile_resort": True}])
def test_options_on_degenerate_inputs(R, dev, opt):
    """Each option with no Gaussians, one Gaussian, a 1x1 image and a view that
    sees nothing: the images are the background, the gradients zero or
    finite, and the statistics arrays untouched where nothing is visible."""
    bg = (0.25, 0.5, 0.75)
    st = _settings(tile=(8, 8), bg=bg, **opt)
    gnorm = torch.zeros(4, dtype=torch.float32, device=dev)
    vcount = torch.zeros(4, dtype=torch.int32, device=dev)
    R.set_densify_stats(gnorm, vcount)
    try:
        cam = scenes.axis_camera(4.0, 9, 7, 40.0)
        back = scenes.Camera(cam.R, np.float32([0, 0, -10.0]), cam.fx, cam.fy, cam.cx, cam.cy,
                             9, 7)                          # every mean behind this camera
        tiny = scenes.axis_camera(4.0, 1, 1, 40.0)
        for n in (0, 1, 4):
            rng = np.random.default_rng(n)
            dens = rng.uniform(0.2, 0.9, n) if opt else rng.uniform(1, 5, n)
            sc = H.scene(rng.uniform(-0.3, 0.3, (n, 3)), np.full((n, 3), 0.2), dens,
                         rgb=rng.uniform(0, 1, (n, 3)))
            t = G.device_scene(sc, dev)
            imgs = R.forward(*t, [cam, back, tiny], st)
            b = imgs[1].cpu().numpy()
            assert np.allclose(b, np.array(bg, np.float32)[:, None, None])
            if n == 0:
                assert np.allclose(imgs[0].cpu().numpy(), np.array(bg, np.float32)[:, None, None])
            grads = [torch.zeros_like(x) for x in t]
            R.backward([torch.ones_like(x) for x in imgs], *grads)
            torch.cuda.synchronize()
            for g in grads:
                assert torch.isfinite(g).all()
        assert int(vcount.sum()) >= 0 and torch.isfinite(gnorm).all()
    finally:
        R.set_densify_stats(None, None)
