"""GPU parity of the per-tile re-sorting (each tile composites in the order
of the depth of every Gaussian's maximum on the tile-centre ray; the
re-sorting the paper points to against popping, Sec. 7) against the FP64
oracle through the C ABI."""
import math

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
    return Settings(tile_resort=True, **kw)


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, bg=st.bg, act=st.act, resort_tile=tuple(st.tile))


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8)])
def test_tile_resort_parity(R, dev, tile):
    """The parity workload (128x128, 1000 Gaussians) with the per-tile order:
    image and gradients; pixels whose order rests on keys closer than
    MARGIN_ORDER (relative) are in the flagged set."""
    wl = scenes.config1()
    sc, cam = wl.scene, wl.cams[0]
    st = _settings(tile=tile, act="softplus", bg=(0.1, 0.2, 0.3))
    ost = _oset(st)
    ref = oracle.render(sc, cam, ost)
    base = oracle.render(sc, cam, oracle.Settings(act="softplus", bg=(0.1, 0.2, 0.3)))
    t = G.device_scene(sc, dev)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    moved = float(np.abs(ref["image"] - base["image"]).max())
    G.check_image(img, ref, label=f"largest change from the mean-depth order {moved:.3g}; ")
    assert moved > 1e-3            # the order matters on this scene
    rng = np.random.default_rng(71)
    dL = G.upstream(rng, ref, 3)
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(dL.astype(np.float32)).to(dev)], *grads)
    torch.cuda.synchronize()
    g = oracle.render_backward(sc, cam, ost, dL)
    G.check_grads({k: gr.cpu().numpy() for k, gr in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward([g], G.GRAD_KEYS))


def test_tile_resort_flips_two_gaussians(R, dev):
    """The long Gaussian whose maximum lies in front of a smaller one with a
    nearer mean is composited first with the option, second without."""
    cam = scenes.axis_camera(0.0, 16, 16, 30.0)    # one 16x16 tile centred on the axis
    phi = -math.pi / 4
    q = [math.cos(phi / 2), 0.0, math.sin(phi / 2), 0.0]
    sc = H.scene([[0.0, 0.0, 4.7], [0.5, 0.0, 5.0]], [[0.08] * 3, [0.6, 0.05, 0.05]], [3.0, 4.0],
                 quats=[[1, 0, 0, 0], q], rgb=[[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    t = G.device_scene(sc, dev)
    from paper_2412_03378_amd import Settings
    for st in (_settings(tile=(16, 16)), Settings(tile=(16, 16))):
        img = R.forward(*t, [cam], st)[0].cpu().numpy()
        ost = _oset(st) if st.tile_resort else oracle.Settings()
        ref = oracle.render(sc, cam, ost)
        assert np.abs(img - ref["image"]).max() <= G.IMG_TOL
    c = 8
    on = R.forward(*t, [cam], _settings(tile=(16, 16)))[0].cpu().numpy()[:, c, c]
    off = R.forward(*t, [cam], Settings(tile=(16, 16)))[0].cpu().numpy()[:, c, c]
    assert on[2] > off[2] and on[0] < off[0]     # blue (the long one) in front with the option


def test_tile_resort_rejects_other_modes(R, dev):
    from paper_2412_03378_amd import _lib as L
    wl = scenes.config1(n=100, width=32, height=32)
    t = G.device_scene(wl.scene, dev)
    for kw in (dict(mode="xray"), dict(alpha_model="splat")):
        with pytest.raises(L.VgrError) as ei:
            R.forward(*t, wl.cams, _settings(tile=(8, 8), **kw))
        assert ei.value.code == L.VGR_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [2000, 9000])
def test_tile_resort_long_lists(R, dev, n):
    """Tile lists longer than one wave's sort (2000 entries: one block sorts
    it in LDS) and than one block's (9000: sorted runs of 4096 merged).
    Large isotropic Gaussians cover the whole 16x16 image, so every tile lists
    all n; their means sit at view depths 6 + i 1e-3 with lateral offsets of
    +-(5 + 1/3) 1e-3 / a along x (a: the tile-centre ray's x slope), so that
    on every tile-centre ray the keys lie on a grid of 1e-3 / 3, distinct and
    further apart than MARGIN_ORDER, in an order that differs from the
    depth order.  Low opacities keep every Gaussian in every pixel's sum:
    image and gradients against the oracle."""
    cam = scenes.axis_camera(4.0, 16, 16, 20.0)
    a = 4.0 / cam.fx
    rng = np.random.default_rng(81 + n)
    delta = 1e-3
    z = 6.0 + delta * np.arange(n)
    sgn = rng.choice([-1.0, 1.0], n)
    x = sgn * (5.0 + 1.0 / 3.0) * delta / a
    means = np.c_[x, np.zeros(n), z - 4.0]          # world = view - (0, 0, 4)
    # reddish on one side, bluish on the other: the re-sorting moves one
    # group forward on each tile, which shows in the image
    rgb = (np.where(sgn[:, None] > 0, [0.9, 0.1, 0.2], [0.1, 0.2, 0.9])
           + rng.uniform(-0.05, 0.05, (n, 3)))
    sigma = 10.0
    alpha = 0.002 if n < 5000 else 0.001
    kappa = alpha / (math.sqrt(2.0 * math.pi) * sigma)
    perm = rng.permutation(n)
    sc = H.scene(means[perm], [[sigma] * 3], [kappa], rgb=rgb[perm])
    st = _settings(tile=(8, 8), alpha_min=1e-4, T_min=1e-6, bg=(0.1, 0.2, 0.3))
    ost = oracle.Settings(alpha_min=st.alpha_min, T_min=st.T_min, bg=st.bg, act=st.act,
                          resort_tile=(8, 8))
    ref = oracle.render(sc, cam, ost)
    base = oracle.render(sc, cam, oracle.Settings(alpha_min=st.alpha_min, T_min=st.T_min,
                                                  bg=st.bg, act=st.act))
    moved = float(np.abs(ref["image"] - base["image"]).max())
    t = G.device_scene(sc, dev)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    G.check_image(img, ref, label=f"n={n}: largest change from the depth order {moved:.3g}; ")
    assert moved > 1e-3            # the order matters on this scene
    assert int((np.asarray(ref["margin_order"]) <= G.MARGIN_ORDER).sum()) == 0
    rng2 = np.random.default_rng(91 + n)
    dL = G.upstream(rng2, ref, 3)
    grads = [torch.zeros_like(v) for v in t]
    R.backward([torch.from_numpy(dL.astype(np.float32)).to(dev)], *grads)
    torch.cuda.synchronize()
    g = oracle.render_backward(sc, cam, ost, dL)
    G.check_grads({k: gr.cpu().numpy() for k, gr in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward([g], G.GRAD_KEYS), label=f"n={n} ")
