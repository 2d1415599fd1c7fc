"""Parity at the full workload sizes, in the launch configuration the
benchmark times, on outputs the FP64 oracle can compute one by one:

* forward: sampled pixels of the full-size render;
* backward: an upstream gradient that is non-zero only at sampled pixels,
  so the exact parameter gradient is the oracle's backward over those pixels.
"""
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


def _settings(**kw):
    from paper_2412_03378_amd import Settings
    return Settings(**kw)


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, x_min_xray=st.x_min_xray, bg=st.bg, act=st.act,
                           density=st.density, alpha_model=st.alpha_model,
                           near_segment=st.near_segment, kernel=st.kernel,
                           resort_tile=tuple(st.tile) if st.tile_resort else None,
                           pixel_window=st.pixel_window)


def _pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    pts = [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (W // 2, H // 2)]
    pts += list(zip(rng.integers(0, W, n).tolist(), rng.integers(0, H, n).tolist()))
    return np.array(pts, np.int32)


def _check_forward(img, T, last, sc, cam, st, pix, xray=False, order_share=None):
    ref = oracle.render(sc, cam, _oset(st), pixels=pix)
    if xray:
        got = img[pix[:, 1], pix[:, 0]][None]
    else:
        got = img[:, pix[:, 1], pix[:, 0]]
    G.check_image(got, ref, xray=xray, label=f"{len(pix)} pixels: ", order_share=order_share)
    ok = G.ok_mask(ref, xray)
    if not xray:
        assert np.abs(T[pix[:, 1], pix[:, 0]] - ref["T"])[ok].max() <= G.IMG_TOL
        assert np.array_equal(last[pix[:, 1], pix[:, 0]][ok], ref["last"][ok])
    return ref


def _sparse_upstream(sc, cams, st, pix_per_view, seed, dev, order_share=None):
    """dL non-zero only at the sampled pixels of each view (unflagged ones in
    colour mode), zero on views without samples; returns the device tensors
    and, per sampled view, (view index, pixels, values)."""
    rng = np.random.default_rng(seed)
    xray = st.mode == "xray"
    nch = 1 if xray else 3
    dLs, sparse = [], []
    for v, cam in enumerate(cams):
        full = np.zeros((nch, cam.height, cam.width), np.float32)
        pix = pix_per_view.get(v)
        if pix is not None:
            ref = oracle.render(sc, cam, _oset(st), pixels=pix)
            keep = pix[G.ok_mask(ref, xray)]
            G.check_flag_share(ref, xray, order_share)
            g = rng.standard_normal((nch, len(keep)))
            full[:, keep[:, 1], keep[:, 0]] = g
            sparse.append((v, keep, g))
        dLs.append(torch.from_numpy(full if nch == 3 else full[0]).to(dev))
    return dLs, sparse


def _oracle_grads(sc, cams, st, sparse, names):
    parts, flips = [], []
    for v, keep, g in sparse:
        parts.append(oracle.render_backward(sc, cams[v], _oset(st), g, pixels=keep))
        if st.mode == "xray":
            flips.append(oracle.render_backward(sc, cams[v], _oset(st), g, pixels=keep,
                                                near_threshold=G.MARGIN_X))
    return G.sum_backward(parts, names, flips or None)


def _sparse_backward(R, dev, t, sc, cams, st, pix_per_view, seed, has_sh, order_share=None):
    """Backward with dL non-zero only at sampled pixels (pix_per_view: a list
    aligned with cams, or a dict view -> pixels)."""
    if not isinstance(pix_per_view, dict):
        pix_per_view = dict(enumerate(pix_per_view))
    R.forward(*t, cams, st)
    dLs, sparse = _sparse_upstream(sc, cams, st, pix_per_view, seed, dev, order_share)
    grads = [torch.zeros_like(x) for x in t[:4]] + [torch.zeros_like(t[4]) if has_sh else None]
    R.backward(dLs, *grads)
    torch.cuda.synchronize()
    names = G.GRAD_KEYS[:5 if has_sh else 4]
    G.check_grads({k: gr.cpu().numpy() for k, gr in zip(names, grads)},
                  _oracle_grads(sc, cams, st, sparse, names))


TILE = (8, 8)


@pytest.fixture(scope="module")
def cfg2(dev):
    wl = scenes.config2(with_grad=False)
    return wl, G.device_scene(wl.scene, dev)


def test_config2_forward_sampled(R, cfg2):
    wl, t = cfg2
    cam = wl.cams[0]
    st = _settings(sh_degree=3, tile=TILE)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    T, last = R.aux(0, cam.height, cam.width)
    G.check_emission(R)
    _check_forward(img, T.cpu().numpy(), last.cpu().numpy(), wl.scene, cam, st,
                   _pixels(cam, 96, 21))


def test_config2_backward_sparse(R, dev, cfg2):
    wl, t = cfg2
    st = _settings(sh_degree=3, tile=TILE)
    _sparse_backward(R, dev, t, wl.scene, wl.cams, st, [_pixels(wl.cams[0], 40, 22)], 23, True)


def test_config2_splat_sampled(R, dev, cfg2):
    """The forward/backward A/B configuration of the benchmark: the headline
    scene with the splatting opacity, peak opacities o = 1 - exp(-kappa
    sqrt(2 pi) (s_x s_y s_z)^(1/3)) as the benchmark sets them."""
    wl, t = cfg2
    sc = wl.scene
    sg = np.cbrt(np.prod(sc.scales.astype(np.float64), axis=1))
    o = (-np.expm1(-sc.dens.astype(np.float64) * np.sqrt(2.0 * np.pi) * sg)).astype(np.float32)
    sc = scenes.Scene(sc.means, sc.quats, sc.scales, o, sc.sh, sc.sh_degree)
    ts = list(t)
    ts[3] = torch.from_numpy(o).to(dev)
    cam = wl.cams[0]
    st = _settings(sh_degree=3, tile=TILE, alpha_model="splat")
    img = R.forward(*ts, [cam], st)[0].cpu().numpy()
    T, last = R.aux(0, cam.height, cam.width)
    _check_forward(img, T.cpu().numpy(), last.cpu().numpy(), sc, cam, st, _pixels(cam, 64, 24))
    _sparse_backward(R, dev, ts, sc, [cam], st, [_pixels(cam, 30, 25)], 26, True)


def test_config2_near_segment_sampled(R, dev, cfg2):
    """The headline scene with the near-plane segment on (the benchmark's
    option-cost configuration: the segment kernels, no record flagged)."""
    wl, t = cfg2
    cam = wl.cams[0]
    st = _settings(sh_degree=3, tile=TILE, near_segment=True)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    T, last = R.aux(0, cam.height, cam.width)
    _check_forward(img, T.cpu().numpy(), last.cpu().numpy(), wl.scene, cam, st,
                   _pixels(cam, 64, 27))
    _sparse_backward(R, dev, t, wl.scene, [cam], st, [_pixels(cam, 30, 28)], 29, True)


# Share of sampled pixels of the headline scene whose order keys (per tile,
# or the per-pixel window's) lie within MARGIN_ORDER of each other: about a
# third at 1080p with 1M clustered Gaussians (26 blended per pixel at the
# median), so the re-sorting options are checked on the other two thirds.
ORDER_SHARE = 0.5


@pytest.mark.parametrize("window", [0, 8])
def test_config2_resort_sampled(R, dev, cfg2, window):
    """The headline scene with the per-tile order, alone and with a per-pixel
    window of 8 (the benchmark's option-cost configurations)."""
    wl, t = cfg2
    cam = wl.cams[0]
    st = _settings(sh_degree=3, tile=TILE, tile_resort=True, pixel_window=window)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    T, last = R.aux(0, cam.height, cam.width)
    G.check_emission(R)
    _check_forward(img, T.cpu().numpy(), last.cpu().numpy(), wl.scene, cam, st,
                   _pixels(cam, 128, 30 + window), order_share=ORDER_SHARE)
    _sparse_backward(R, dev, t, wl.scene, [cam], st, [_pixels(cam, 60, 31 + window)], 32 + window,
                     True, order_share=ORDER_SHARE)


@pytest.mark.parametrize("tile", [TILE, (16, 16)])   # 16x16: the shape the benchmark's tuner picks
def test_config4_xray_sampled(R, dev, tile):
    wl = scenes.config4(with_grad=False)
    t = G.device_scene(wl.scene, dev)
    st = _settings(mode="xray", tile=tile, x_min_xray=scenes.XRAY_X_MIN)
    imgs = R.forward(*t, wl.cams, st)
    G.check_emission(R)
    for v in (0, 21, 42, 63):
        _check_forward(imgs[v].cpu().numpy(), None, None, wl.scene, wl.cams[v], st,
                       _pixels(wl.cams[v], 24, 40 + v), xray=True)
    cams = [wl.cams[5], wl.cams[37]]
    _sparse_backward(R, dev, t, wl.scene, cams, st, [_pixels(c, 16, 50 + k) for k, c in
                                                      enumerate(cams)], 51, False)


@pytest.mark.parametrize("tile", [TILE, (16, 16)])   # 16x16: the benchmark's tuned shape
def test_config3_batched_sampled(R, dev, tile):
    wl = scenes.config3(with_grad=False)
    t = G.device_scene(wl.scene, dev)
    st = _settings(sh_degree=3, tile=tile)
    imgs = [x.cpu().numpy() for x in R.forward(*t, wl.cams, st)]
    G.check_emission(R)
    for v in (0, 7, 15):
        T, last = R.aux(v, wl.cams[v].height, wl.cams[v].width)
        _check_forward(imgs[v], T.cpu().numpy(), last.cpu().numpy(), wl.scene, wl.cams[v], st,
                       _pixels(wl.cams[v], 16, 60 + v))
    for v in (3, 12):
        one = R.forward(*t, [wl.cams[v]], st)[0].cpu().numpy()
        assert np.array_equal(one, imgs[v])


@pytest.fixture(scope="module")
def cfg3(dev):
    wl = scenes.config3(with_grad=False)
    return wl, G.device_scene(wl.scene, dev)


def test_config3_backward_sparse(R, dev, cfg3):
    """The benchmark's batched step: all 16 views of mixed resolution in one
    forward + backward at 16x16 tiles, SH3; upstream gradients at sampled
    pixels of four views spread over the batch."""
    wl, t = cfg3
    st = _settings(sh_degree=3, tile=(16, 16))
    pix = {v: _pixels(wl.cams[v], 8, 80 + v) for v in (0, 5, 10, 15)}
    _sparse_backward(R, dev, t, wl.scene, wl.cams, st, pix, 81, True)


def test_config3_graph_replay_against_oracle(dev, cfg3):
    """The same step captured as one hipGraph: the second replay's images at
    sampled pixels and its gradients against the oracle (not only against an
    eager call)."""
    from paper_2412_03378_amd import Renderer
    wl, t = cfg3
    sc, cams = wl.scene, wl.cams
    st = _settings(sh_degree=3, tile=(16, 16))
    pix = {v: _pixels(cams[v], 6, 90 + v) for v in (2, 9, 14)}
    dLs, sparse = _sparse_upstream(sc, cams, st, pix, 91, dev)
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in cams]
    grads = [torch.zeros_like(x) for x in t]
    r = Renderer(0)
    try:
        r.graph_capture(list(t), cams, st, outs, dLs, grads, capacity_factor=1.25, zero_grads=True)
        for _ in range(2):
            for o in outs:
                o.fill_(-1.0)
            for gr in grads:
                gr.fill_(7.0)
            r.graph_launch()
            r.graph_check()
        imgs = [o.cpu().numpy() for o in outs]
        for v, p in pix.items():
            ref = oracle.render(sc, cams[v], _oset(st), pixels=p)
            G.check_image(imgs[v][:, p[:, 1], p[:, 0]], ref, label=f"graph view {v}: ")
        G.check_grads({k: gr.cpu().numpy() for k, gr in zip(G.GRAD_KEYS, grads)},
                      _oracle_grads(sc, cams, st, sparse, G.GRAD_KEYS))
    finally:
        r.close()


@pytest.mark.parametrize("tile,views", [(TILE, (0, 33)), ((16, 16), tuple(range(16)))])
def test_config5_views_sampled(R, dev, tile, views):
    """Two views at 8x8, and the benchmark's training call: 16 views in one
    call at its tuned 16x16 tiles (two of them checked)."""
    wl = scenes.config5(with_grad=False)
    t = G.device_scene(wl.scene, dev)
    st = _settings(sh_degree=3, tile=tile)
    cams = [wl.cams[v] for v in views]
    imgs = [x.cpu().numpy() for x in R.forward(*t, cams, st)]
    G.check_emission(R)
    for v in (0, len(cams) - 1):
        cam = cams[v]
        T, last = R.aux(v, cam.height, cam.width)
        _check_forward(imgs[v], T.cpu().numpy(), last.cpu().numpy(), wl.scene, cam, st,
                       _pixels(cam, 12, 70 + v))
    if len(cams) == 16:
        # the training call's backward (16 views, 6M Gaussians, SH3), upstream
        # gradients at sampled pixels of three views
        del imgs
        pix = {v: _pixels(cams[v], 6, 100 + v) for v in (1, 8, 14)}
        _sparse_backward(R, dev, t, wl.scene, cams, st, pix, 101, True)
