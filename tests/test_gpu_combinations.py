"""Seeded random combinations of every rendering setting (mode, SH degree,
activation, density input, opacity model, near-plane segment, kernel,
re-sorting and its window, tile and batch shape, thresholds, background,
one to three views of uneven size) on small scenes, each against the FP64
oracle through the C ABI: images and gradients, with the same margin and
tolerance rules as the other parity tests."""
import numpy as np
import pytest

import oracle
import gpu_helpers as G
from paper_2412_03378_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILES = [(8, 8), (16, 8), (16, 16), (32, 8)]
N_CASES = 64


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def R(dev):
    from paper_2412_03378_amd import Renderer
    return Renderer(0)


def _draw(seed):
    """One valid combination of settings, its scene and cameras."""
    from paper_2412_03378_amd import Settings
    rng = np.random.default_rng(1000 + seed)
    pick = lambda xs: xs[int(rng.integers(len(xs)))]
    mode = pick(["color", "color", "xray"])
    colour = mode == "color"
    alpha_model = pick(["volumetric", "volumetric", "splat"]) if colour else "volumetric"
    vol = alpha_model == "volumetric"
    kernel = pick(["gaussian", "gaussian", "epanechnikov"]) if vol else "gaussian"
    near = bool(vol and kernel == "gaussian" and rng.random() < 0.3)
    density = pick(["kappa", "theta"]) if alpha_model == "volumetric" else "kappa"
    resort = bool(colour and vol and rng.random() < 0.3)
    window = int(rng.integers(1, 9)) if (resort and rng.random() < 0.5) else 0
    tile = (8, 8) if window else pick(TILES)
    batch = 64 if window else pick([32, 64])
    deg = int(rng.integers(0, 4)) if colour else 0
    st = Settings(mode=mode, sh_degree=deg, act=pick(["clamp", "softplus"]),
                  alpha_min=pick([1.0 / 255.0, 0.01]), alpha_max=pick([0.99, 0.9]),
                  T_min=pick([1e-4, 0.05]), x_min_xray=pick([1e-6, 1e-4]),
                  bg=tuple(float(v) for v in rng.uniform(0, 0.4, 3)), tile=tile, batch=batch,
                  density=density, alpha_model=alpha_model, near_segment=near,
                  tile_resort=resort, kernel=kernel, pixel_window=window)
    n = int(rng.integers(150, 500))
    means = rng.uniform(-1.0, 1.0, (n, 3))
    lo, hi = (0.03, 0.25) if kernel == "epanechnikov" else (0.01, 0.15)
    s = np.exp(rng.uniform(np.log(lo), np.log(hi), (n, 3)))
    q = rng.standard_normal((n, 4))
    if alpha_model == "splat":
        dens = rng.uniform(0.05, 1.0, n)
    elif density == "theta":
        dens = rng.uniform(0.02, 0.98, n)
    else:
        dens = np.exp(rng.uniform(np.log(0.2), np.log(15.0), n))
    sh = rng.normal(0.0, 0.3, (n, (deg + 1) ** 2, 3))
    sh[:, 0, :] = (rng.uniform(0, 1, (n, 3)) - 0.5) / scenes.Y00
    sc = scenes.Scene(np.float32(means), np.float32(q), np.float32(s), np.float32(dens),
                      np.float32(sh), deg)
    cams = []
    for v in range(int(rng.integers(1, 4))):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        dist = rng.uniform(3.0, 4.5)
        w, h = int(rng.integers(24, 73)), int(rng.integers(20, 61))
        c = scenes.look_at(dist * d, (0, 0, 0), w, h, float(rng.uniform(40, 65)))
        # the near plane cuts the scene's cube: Gaussians straddle it
        cams.append(scenes.Camera(c.R, c.t, c.fx, c.fy, c.cx, c.cy, c.width, c.height,
                                  znear=float(dist - 0.8)))
    return st, sc, cams


def _oset(st):
    return oracle.Settings(mode=st.mode, alpha_min=st.alpha_min, alpha_max=st.alpha_max,
                           T_min=st.T_min, x_min_xray=st.x_min_xray, bg=st.bg, act=st.act,
                           density=st.density, alpha_model=st.alpha_model,
                           near_segment=st.near_segment, kernel=st.kernel,
                           resort_tile=tuple(st.tile) if st.tile_resort else None,
                           pixel_window=st.pixel_window)


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_combination(R, dev, case):
    st, sc, cams = _draw(case)
    label = (f"case {case}: {st.mode} deg {st.sh_degree} {st.act} {st.density} {st.alpha_model} "
             f"near {st.near_segment} {st.kernel} resort {st.tile_resort} window {st.pixel_window} "
             f"tile {st.tile} batch {st.batch} views {len(cams)} n {sc.n}; ")
    print(label, flush=True)
    xray = st.mode == "xray"
    nch = 1 if xray else 3
    ost = _oset(st)
    t = G.device_scene(sc, dev)
    if xray:
        t = t[:4] + (None,)
    imgs = R.forward(*t, cams, st)
    G.check_emission(R)
    refs = [oracle.render(sc, c, ost) for c in cams]
    for v, (img, ref) in enumerate(zip(imgs, refs)):
        img = img.cpu().numpy()
        G.check_image(img[None] if xray else img, ref, xray=xray, label=f"{label}view {v}: ")
    rng = np.random.default_rng(5000 + case)
    dLs = [G.upstream(rng, ref, nch, xray) for ref in refs]
    keys = G.GRAD_KEYS[:4] if xray else G.GRAD_KEYS
    grads = [torch.zeros_like(x) for x in t[:4]] + ([None] if xray else [torch.zeros_like(t[4])])
    R.backward([torch.from_numpy((d[0] if xray else d).astype(np.float32)).to(dev) for d in dLs],
               *grads)
    torch.cuda.synchronize()
    parts = [oracle.render_backward(sc, c, ost, d) for c, d in zip(cams, dLs)]
    flips = ([oracle.render_backward(sc, c, ost, d, near_threshold=G.MARGIN_X)
              for c, d in zip(cams, dLs)] if xray else None)
    G.check_grads({k: g.cpu().numpy() for k, g in zip(keys, grads)},
                  G.sum_backward(parts, keys, flips), label=label)
