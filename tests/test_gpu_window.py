"""GPU parity of the per-pixel re-sorting window (the per-pixel level of the
re-sorting the paper points to against popping, Sec. 7, Limitations): each
pixel's Gaussians, in the per-tile order, pass through a window of W entries
ordered by the depth of each maximum on the pixel's own ray.  Against the
FP64 oracle through the C ABI."""
import numpy as np
import pytest

import oracle
import gpu_helpers as G
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


def _settings(W, **kw):
    from paper_2412_03378_amd import Settings
    kw.setdefault("act", "softplus")
    kw.setdefault("bg", (0.1, 0.2, 0.3))
    return Settings(tile_resort=True, tile=(8, 8), pixel_window=W, **kw)


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, bg=st.bg, act=st.act, resort_tile=(8, 8),
                           pixel_window=st.pixel_window, near_segment=st.near_segment,
                           kernel=st.kernel)


def _check(R, dev, sc, cams, st, seed, label=""):
    """Forward and backward of all views in one call against the oracle."""
    ost = _oset(st)
    refs = [oracle.render(sc, c, ost) for c in cams]
    t = G.device_scene(sc, dev)
    imgs = R.forward(*t, cams, st)
    for v, (img, ref) in enumerate(zip(imgs, refs)):
        G.check_image(img.cpu().numpy(), ref, label=f"{label}view {v}: ")
    G.check_emission(R)
    rng = np.random.default_rng(seed)
    dLs = [G.upstream(rng, ref, 3) for ref in refs]
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(d.astype(np.float32)).to(dev) for d in dLs], *grads)
    torch.cuda.synchronize()
    parts = [oracle.render_backward(sc, c, ost, d) for c, d in zip(cams, dLs)]
    G.check_grads({k: g.cpu().numpy() for k, g in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward(parts, G.GRAD_KEYS), label=label)
    return imgs


@pytest.mark.parametrize("W", [1, 2, 3, 4, 8, 16, 32])
def test_window_parity(R, dev, W):
    """The parity workload (128x128, 1000 Gaussians) with windows of every
    register size class: image and gradients; pixels whose order rests on
    keys closer than MARGIN_ORDER (per-tile or per-pixel) are flagged."""
    wl = scenes.config1()
    _check(R, dev, wl.scene, wl.cams, _settings(W), 90 + W, label=f"W={W} ")


def test_window_changes_the_order(R, dev):
    """On the parity workload a long window moves pixels away from the
    per-tile order (so the parity above tests the window), and W = 1 is the
    per-tile order bit for bit, forward and backward."""
    from paper_2412_03378_amd import Settings
    wl = scenes.config1()
    sc, cam = wl.scene, wl.cams[0]
    t = G.device_scene(sc, dev)
    tile = Settings(tile_resort=True, tile=(8, 8), act="softplus", bg=(0.1, 0.2, 0.3))
    a = R.forward(*t, [cam], tile)[0].cpu().numpy()
    rng = np.random.default_rng(5)
    dL = torch.from_numpy(rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)).to(dev)
    ga = [torch.zeros_like(x) for x in t]
    R.backward([dL], *ga)
    b = R.forward(*t, [cam], _settings(1))[0].cpu().numpy()
    gb = [torch.zeros_like(x) for x in t]
    R.backward([dL], *gb)
    torch.cuda.synchronize()
    assert np.array_equal(a, b)
    for x, y in zip(ga, gb):
        # gradient sums use FP32 atomics: equal up to the order of additions
        assert torch.allclose(x, y, rtol=1e-4, atol=1e-6 * float(y.abs().max()))
    w = R.forward(*t, [cam], _settings(32))[0].cpu().numpy()
    ref_w = oracle.render(sc, cam, _oset(_settings(32)))["image"]
    ref_t = oracle.render(sc, cam, _oset(_settings(1)))["image"]
    moved = float(np.abs(ref_w - ref_t).max())
    print(f"largest change from the per-tile order {moved:.3g}")
    assert moved > 1e-3
    assert float(np.abs(w - a).max()) > 1e-3


@pytest.mark.parametrize("T_min", [0.05, 0.3])
def test_window_termination(R, dev, T_min):
    """Early termination with entries still in the window (they are not
    composited): a dense scene and a high T_min."""
    wl = scenes.config1(n=2000, width=96, height=80, seed=7)
    _check(R, dev, wl.scene, wl.cams, _settings(8, T_min=T_min), 120, label=f"T_min={T_min} ")


@pytest.mark.parametrize("opt", ["near", "epan"])
def test_window_with_options(R, dev, opt):
    """The window with the near-plane segment (the plane through the scene,
    so Gaussians straddle it) and with the Epanechnikov kernel."""
    if opt == "near":
        wl = scenes.config1(n=800, width=96, height=96, seed=11)
        c = scenes.axis_camera(4.0, 96, 96, 60.0)
        # the near plane at world z = -0.8 cuts through the scene's cube
        cam = scenes.Camera(c.R, c.t, c.fx, c.fy, c.cx, c.cy, c.width, c.height, znear=3.2)
        _check(R, dev, wl.scene, [cam], _settings(4, near_segment=True), 130, label="near ")
    else:
        wl = scenes.config1(n=800, width=96, height=96, seed=12)
        _check(R, dev, wl.scene, wl.cams, _settings(4, kernel="epanechnikov"), 131, label="epan ")


def test_window_batched_views_and_reuse(R, dev):
    """Three views of different sizes in one call, then a smaller call on the
    same context (pair slots left by the first call must not leak into the
    second)."""
    wl = scenes.config1(n=1500, seed=21)
    cams = [scenes.look_at([0.5, -0.4, -4.0], (0, 0, 0), 120, 88, 55.0),
            scenes.look_at([-3.5, 0.6, -2.0], (0, 0, 0), 64, 72, 50.0),
            scenes.look_at([2.0, 2.5, -3.0], (0, 0, 0), 40, 40, 60.0)]
    _check(R, dev, wl.scene, cams, _settings(6), 140, label="3 views ")
    small = scenes.config1(n=300, width=48, height=40, seed=22)
    _check(R, dev, small.scene, small.cams, _settings(6), 141, label="after ")


def test_window_graph_replay(dev):
    """A captured forward + backward with the window replays to the eager
    result (several replays, with unrelated eager work and syncs between)."""
    from paper_2412_03378_amd import Renderer
    wl = scenes.config1(n=1000, seed=31)
    sc, cams = wl.scene, wl.cams
    st = _settings(8)
    t = G.device_scene(sc, dev)
    rng = np.random.default_rng(32)
    dL = [torch.from_numpy(rng.standard_normal((3, c.height, c.width)).astype(np.float32)).to(dev)
          for c in cams]
    r0 = Renderer(0)
    eager = [x.clone() for x in r0.forward(*t, cams, st)]
    ge = [torch.zeros_like(x) for x in t]
    r0.backward(dL, *ge)
    torch.cuda.synchronize()
    r = Renderer(0)
    outs = [torch.empty_like(e) for e in eager]
    gg = [torch.zeros_like(x) for x in t]
    r.graph_capture(t, cams, st, outs, dL, gg, capacity_factor=1.25, zero_grads=True)
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        r.graph_launch()
        r.graph_check()
        junk = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep
        for a, b in zip(gg, ge):
            # gradient sums use FP32 atomics: equal up to the order of additions
            assert torch.allclose(a, b, rtol=1e-4, atol=1e-6 * float(b.abs().max())), rep


def test_window_rejects(R, dev):
    from paper_2412_03378_amd import _lib as L, Settings
    wl = scenes.config1(n=100, width=32, height=32)
    t = G.device_scene(wl.scene, dev)
    bad = [Settings(pixel_window=4, tile=(8, 8)),                       # no per-tile order
           Settings(tile_resort=True, pixel_window=4, tile=(16, 16)),
           Settings(tile_resort=True, pixel_window=4, tile=(8, 8), batch=32),
           Settings(tile_resort=True, pixel_window=L.VGR_MAX_PIXEL_WINDOW + 1, tile=(8, 8)),
           Settings(tile_resort=True, pixel_window=-1, tile=(8, 8))]
    for st in bad:
        with pytest.raises(L.VgrError) as ei:
            R.forward(*t, wl.cams, st)
        assert ei.value.code == L.VGR_ERR_INVALID_ARG


def test_window_edge_cases(R, dev):
    """No Gaussians (background, zero gradients), an image smaller than one
    tile, and the rejected X-ray combination."""
    from paper_2412_03378_amd import _lib as L, Settings
    st = _settings(4)
    empty = scenes.config1(n=1, width=20, height=12, seed=41)
    t = [x[:0].contiguous() for x in G.device_scene(empty.scene, dev)]
    img = R.forward(*t, empty.cams, st)[0].cpu().numpy()
    assert np.allclose(img, np.asarray(st.bg, np.float32)[:, None, None])
    small = scenes.config1(n=300, width=5, height=3, seed=42)
    _check(R, dev, small.scene, small.cams, st, 150, label="5x3 ")
    with pytest.raises(L.VgrError) as ei:
        R.forward(*G.device_scene(small.scene, dev), small.cams,
                  Settings(mode="xray", tile_resort=True, tile=(8, 8), pixel_window=4))
    assert ei.value.code == L.VGR_ERR_INVALID_ARG


def test_window_through_autograd(dev):
    """render() with a window: the autograd gradients equal the explicit
    backward of the same call."""
    from paper_2412_03378_amd import Renderer, render
    wl = scenes.config1(n=600, width=64, height=48, seed=43)
    st = _settings(8)
    base = G.device_scene(wl.scene, dev)
    leaves = [x.clone().requires_grad_(True) for x in base]
    imgs = render(*leaves, wl.cams, st)
    rng = np.random.default_rng(44)
    dL = torch.from_numpy(rng.standard_normal(imgs[0].shape).astype(np.float32)).to(dev)
    (imgs[0] * dL).sum().backward()
    r = Renderer(0)
    r.forward(*base, wl.cams, st)
    grads = [torch.zeros_like(x) for x in base]
    r.backward([dL], *grads)
    torch.cuda.synchronize()
    for a, b in zip(leaves, grads):
        assert torch.allclose(a.grad, b, rtol=1e-4, atol=1e-6 * float(b.abs().max()))
