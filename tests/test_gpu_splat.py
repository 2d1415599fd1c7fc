"""GPU parity of the comparison model: the 3DGS splatting opacity (Sec. 3,
eq. 3dgs_alpha, eq. affine_approx) rendered by the same pipeline, against the
FP64 oracle through the C ABI."""
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
    return Settings(alpha_model="splat", **kw)


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, bg=st.bg, act=st.act, alpha_model="splat")


def _check_views(R, dev, sc, cams, st):
    t = G.device_scene(sc, dev)
    imgs = R.forward(*t, cams, st)
    out = []
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, _oset(st))
        img = imgs[v].cpu().numpy()
        G.check_image(img, ref, label=f"view {v} {cam.width}x{cam.height} mean {img.mean():.4f}: ")
        assert np.abs(img - ref["image"]).max() > 0 or img.max() > 0
        out.append(img)
    return out


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (16, 16), (32, 8)])
def test_splat_forward_parity(R, dev, tile):
    """128x128, 1000 Gaussians with peak opacities in [0.05, 1]: every tile
    shape matches the oracle, and the image does not depend on the tile."""
    wl = scenes.config1()
    sc = scenes.with_opacity(wl.scene, seed=51)
    st = _settings(tile=tile, bg=(0.1, 0.2, 0.3))
    img = _check_views(R, dev, sc, wl.cams, st)[0]
    base = R.forward(*G.device_scene(sc, dev), wl.cams, _settings(tile=(8, 8), bg=(0.1, 0.2, 0.3)))
    assert np.array_equal(img, base[0].cpu().numpy())


def test_splat_multi_view_sh3(R, dev):
    """Three views of uneven size in one call, SH degree 3, softplus colour
    (the multi-view preprocess with the splat record)."""
    wl = scenes.config3(n=1500, n_views=3, n_clusters=24, seed=52, with_grad=False)
    sc = scenes.with_opacity(wl.scene, seed=53)
    cams = [scenes.Camera(c.R, c.t, c.fx / 16, c.fy / 16, c.cx / 16, c.cy / 16,
                          c.width // 16, c.height // 16) for c in wl.cams]
    _check_views(R, dev, sc, cams, _settings(sh_degree=3, act="softplus", tile=(16, 8)))


def test_splat_large_off_axis(R, dev):
    """Large anisotropic Gaussians near the image border (the Jacobian's
    depth column dominates their splats), opaque ones clamped at alpha_max,
    and near-plane culls, over a field of small ones."""
    rng = np.random.default_rng(54)
    cam = scenes.axis_camera(4.0, 60, 44, 70.0)
    n_big = 12
    means = np.c_[rng.uniform(-2.2, 2.2, (n_big, 2)), rng.uniform(-1.0, 1.5, n_big)]
    scales = np.c_[rng.uniform(0.05, 0.3, (n_big, 2)), rng.uniform(0.3, 1.0, n_big)]
    means = np.r_[means, [[0.1, 0.0, -3.81], [0.0, 0.1, -3.7]],
                  np.c_[rng.uniform(-1, 1, (200, 2)), rng.uniform(-1, 1, 200)]]
    scales = np.r_[scales, [[0.2] * 3, [0.05] * 3],
                   np.exp(rng.uniform(np.log(0.01), np.log(0.1), (200, 3)))]
    n = means.shape[0]
    op = rng.uniform(0.05, 1.0, n)
    op[:3] = 1.0
    sc = H.scene(means, scales, op, quats=rng.standard_normal((n, 4)),
                 rgb=rng.uniform(0, 1, (n, 3)))
    _check_views(R, dev, sc, [cam], _settings(tile=(8, 8)))


def _grad_check(R, dev, sc, cams, st, seed):
    """Backward of the sum of the views' losses against the oracle's analytic
    splatting backward (pixels with a decision at a threshold get a zero
    upstream gradient)."""
    ost = _oset(st)
    t = G.device_scene(sc, dev)
    R.forward(*t, cams, st)
    rng = np.random.default_rng(seed)
    dLs, refs = [], []
    for cam in cams:
        ref = oracle.render(sc, cam, ost)
        dLs.append(G.upstream(rng, ref, 3))
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(d.astype(np.float32)).to(dev) for d in dLs], *grads)
    torch.cuda.synchronize()
    per = [oracle.render_backward(sc, cam, ost, d) for cam, d in zip(cams, dLs)]
    G.check_grads({k: g.cpu().numpy() for k, g in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward(per, G.GRAD_KEYS))


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_splat_backward_parity(R, dev, tile):
    """Gradients of the splatting model (through Sigma'^-1, the projection
    Jacobian, rotation, scales, opacity and colour) on the parity workload."""
    wl = scenes.config1()
    sc = scenes.with_opacity(wl.scene, seed=56)
    _grad_check(R, dev, sc, wl.cams, _settings(tile=tile, act="softplus", bg=(0.1, 0.2, 0.3)),
                seed=57)


def test_splat_backward_multi_view_sh3(R, dev):
    wl = scenes.config3(n=1500, n_views=3, n_clusters=24, seed=58, with_grad=False)
    sc = scenes.with_opacity(wl.scene, seed=59)
    cams = [scenes.Camera(c.R, c.t, c.fx / 16, c.fy / 16, c.cx / 16, c.cy / 16,
                          c.width // 16, c.height // 16) for c in wl.cams]
    _grad_check(R, dev, sc, cams, _settings(sh_degree=3, act="softplus", tile=(16, 8)), seed=60)


def test_splat_rejects_other_modes(R, dev):
    from paper_2412_03378_amd import _lib as L
    wl = scenes.config1(n=100, width=32, height=32)
    sc = scenes.with_opacity(wl.scene, seed=55)
    t = G.device_scene(sc, dev)
    for kw in (dict(mode="xray"), dict(density="theta")):
        with pytest.raises(L.VgrError) as ei:
            R.forward(*t, wl.cams, _settings(tile=(8, 8), **kw))
        assert ei.value.code == L.VGR_ERR_INVALID_ARG
