"""The rasterisers with 32-record batches (the block-shape dimension the
autotuner sweeps next to the tile shape) against the FP64 oracle, and bitwise
against 64-record batches where the order of work cannot change a result
(forward images)."""
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


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (16, 16), (32, 8)])
def test_batch32_forward_equals_batch64_and_oracle(R, dev, tile):
    wl = scenes.config1()
    sc, cam = wl.scene, wl.cams[0]
    t = G.device_scene(sc, dev)
    a = R.forward(*t, [cam], _settings(tile=tile, batch=32, bg=(0.1, 0.2, 0.3)))[0].cpu().numpy()
    G.check_emission(R)
    b = R.forward(*t, [cam], _settings(tile=tile, batch=64, bg=(0.1, 0.2, 0.3)))[0].cpu().numpy()
    assert np.array_equal(a, b)
    ref = oracle.render(sc, cam, oracle.Settings(bg=(0.1, 0.2, 0.3)))
    G.check_image(a, ref, label=f"tile {tile} batch 32: ")


@pytest.mark.parametrize("tile,mode,kernel", [((8, 8), "color", "gaussian"),
                                               ((16, 16), "color", "gaussian"),
                                               ((8, 8), "xray", "gaussian"),
                                               ((16, 16), "xray", "gaussian"),
                                               ((8, 8), "color", "epanechnikov")])
def test_batch32_backward_against_oracle(R, dev, tile, mode, kernel):
    xray = mode == "xray"
    if xray:
        wl = scenes.config4(n=3000, n_views=64, size=80, seed=4, with_grad=False)
        sc = wl.scene
        cams = [wl.cams[k] for k in (0, 21)]
    else:
        wl = scenes.config1(n=600, width=72, height=60, seed=11)
        sc, cams = wl.scene, wl.cams
        if kernel == "epanechnikov":
            sc = scenes.Scene(sc.means, sc.quats, np.float32(sc.scales * 3.0), sc.dens, sc.sh, 0)
    st = _settings(mode=mode, tile=tile, batch=32, act="softplus", kernel=kernel)
    ost = oracle.Settings(mode=mode, act="softplus", kernel=kernel)
    t = G.device_scene(sc, dev)
    imgs = R.forward(*t, cams, st)
    rng = np.random.default_rng(15)
    dLs = []
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, ost)
        img = imgs[v].cpu().numpy()
        G.check_image(img[None] if xray else img, ref, xray=xray, label=f"view {v}: ")
        dLs.append(G.upstream(rng, ref, 1 if xray else 3, xray))
    keys = G.GRAD_KEYS[:4] if xray else G.GRAD_KEYS
    grads = [torch.zeros_like(x) for x in t[:len(keys)]]
    R.backward([torch.from_numpy((d[0] if xray else d).astype(np.float32)).to(dev) for d in dLs],
               *grads, *([None] if xray else []))
    torch.cuda.synchronize()
    parts = [oracle.render_backward(sc, cam, ost, d) for cam, d in zip(cams, dLs)]
    flips = ([oracle.render_backward(sc, cam, ost, d, near_threshold=G.MARGIN_X)
              for cam, d in zip(cams, dLs)] if xray else None)
    G.check_grads({k: g.cpu().numpy() for k, g in zip(keys, grads)},
                  G.sum_backward(parts, keys, flips))


def test_bad_batch_rejected(R, dev):
    from paper_2412_03378_amd import _lib as L
    wl = scenes.config1(n=20, width=16, height=16)
    t = G.device_scene(wl.scene, dev)
    with pytest.raises(L.VgrError) as e:
        R.forward(*t, wl.cams, _settings(batch=48))
    assert e.value.code == L.VGR_ERR_INVALID_ARG
