"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Sizes: the oracle-sized workloads (128x128 / 1k Gaussians and smaller crops)
span many tiles and ragged edge tiles; the full-size workloads are checked on
sampled pixels in test_gpu_fullsize.py.
"""
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
                           T_min=st.T_min, x_min_xray=st.x_min_xray, bg=st.bg, act=st.act)


# ------------------------------------------------------------------ sort ---

@pytest.mark.parametrize("n,bits,kind", [
    (1, 8, "random"), (4095, 13, "random"), (4096, 13, "random"), (100003, 13, "random"),
    (262144, 32, "random"), (50000, 20, "equal"), (70001, 16, "sorted"),
    (70001, 16, "reversed"), (33333, 32, "max"), (65536, 7, "random"), (0, 8, "random"),
    (4194304, 15, "random"), (4194305, 15, "random"), (6000001, 32, "random"),
    (1000000, 32, "narrow"), (3000000, 24, "narrow")])
def test_radix_sort_stable(R, dev, n, bits, kind):
    rng = np.random.default_rng(n + bits)
    hi = (1 << bits) - 1
    if kind == "random":
        k = rng.integers(0, hi + 1, n, dtype=np.uint64)
    elif kind == "equal":
        k = np.full(n, 12345 & hi, np.uint64)
    elif kind == "sorted":
        k = np.sort(rng.integers(0, hi + 1, n, dtype=np.uint64))
    elif kind == "reversed":
        k = np.sort(rng.integers(0, hi + 1, n, dtype=np.uint64))[::-1].copy()
    elif kind == "narrow":
        # the upper bits are the same for every key (passes over them only copy)
        k = (np.uint64(0x5A) << np.uint64(bits - 8)) | rng.integers(0, 1 << 12, n, dtype=np.uint64)
    else:
        k = np.full(n, hi, np.uint64)
        k[::7] = 0
    k = k.astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(k.view(np.int32)).to(dev)
    vt = torch.from_numpy(v.view(np.int32)).to(dev)
    R.sort_pairs(kt, vt, bits)
    torch.cuda.synchronize()
    order = np.argsort(k, kind="stable")
    assert np.array_equal(kt.cpu().numpy().view(np.uint32), k[order])
    assert np.array_equal(vt.cpu().numpy().view(np.uint32), v[order])


# ------------------------------------------------------- config 1 forward ---

@pytest.fixture(scope="module")
def cfg1():
    return scenes.config1()


@pytest.fixture(scope="module")
def cfg1_ref(cfg1):
    return oracle.render(cfg1.scene, cfg1.cams[0], oracle.Settings())


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_config1_forward(R, dev, cfg1, cfg1_ref, tile):
    sc, cam = cfg1.scene, cfg1.cams[0]
    st = _settings(tile=tile)
    img = R.forward(*G.device_scene(sc, dev), [cam], st)[0]
    T, last = R.aux(0, cam.height, cam.width)
    torch.cuda.synchronize()
    G.check_image(img.cpu().numpy(), cfg1_ref, label=f"tile {tile}: ")
    G.check_emission(R)
    ok = G.ok_mask(cfg1_ref)
    assert np.abs(T.cpu().numpy() - cfg1_ref["T"])[ok].max() <= G.IMG_TOL
    assert np.array_equal(last.cpu().numpy()[ok], cfg1_ref["last"][ok])


def test_tile_shape_independence(R, dev, cfg1):
    sc, cam = cfg1.scene, cfg1.cams[0]
    base = None
    for tile in [(16, 16), (8, 8), (16, 8), (32, 8)]:
        img = R.forward(*G.device_scene(sc, dev), [cam], _settings(tile=tile))[0].cpu().numpy()
        if base is None:
            base = img
        else:
            assert np.abs(img - base).max() <= 1e-6


def test_forward_deterministic(R, dev, cfg1):
    sc, cam = cfg1.scene, cfg1.cams[0]
    a = R.forward(*G.device_scene(sc, dev), [cam], _settings())[0].cpu().numpy()
    b = R.forward(*G.device_scene(sc, dev), [cam], _settings())[0].cpu().numpy()
    assert np.array_equal(a, b)


# ------------------------------------------------------ config 1 backward ---

@pytest.mark.parametrize("act,tile", [("clamp", (16, 16)), ("softplus", (8, 8)), ("clamp", (32, 8))])
def test_config1_backward(R, dev, cfg1, act, tile):
    sc, cam = cfg1.scene, cfg1.cams[0]
    st = _settings(act=act, tile=tile, bg=(0.1, 0.2, 0.3))
    ost = _oset(st)
    ref = oracle.render(sc, cam, ost)
    rng = np.random.default_rng(5)
    dL = G.upstream(rng, ref, 3)
    gref = oracle.render_backward(sc, cam, ost, dL)
    t = G.device_scene(sc, dev)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    G.check_image(img, ref)
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(dL.astype(np.float32)).to(dev)], *grads)
    torch.cuda.synchronize()
    G.check_grads({k: g.cpu().numpy() for k, g in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward([gref], G.GRAD_KEYS))


# ------------------------------------------------------------- X-ray mode ---

def _xray_small(n=3000, size=96, views=3, seed=4):
    wl = scenes.config4(n=n, n_views=64, size=size, seed=seed, with_grad=False)
    return wl.scene, [wl.cams[k] for k in (0, 16, 40)][:views]


# 8x8 tiles: the backward reuses the forward's pre-test masks (one pixel per
# lane); 16x16: it runs its own pre-test
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_xray_forward_backward(R, dev, tile):
    sc, cams = _xray_small()
    st = _settings(mode="xray", tile=tile)
    ost = _oset(st)
    t = G.device_scene(sc, dev)
    imgs = R.forward(*t, cams, st)
    rng = np.random.default_rng(9)
    dLs = []
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, ost)
        # every pixel, the ones with a decision near the cut included
        G.check_image(imgs[v].cpu().numpy()[None], ref, xray=True, label=f"view {v}: ")
        dLs.append(G.upstream(rng, ref, 1, xray=True)[0])
    grads = [torch.zeros_like(x) for x in t[:4]]
    R.backward([torch.from_numpy(d.astype(np.float32)).to(dev) for d in dLs], *grads, None)
    torch.cuda.synchronize()
    keys = G.GRAD_KEYS[:4]
    parts = [oracle.render_backward(sc, cam, ost, d[None]) for cam, d in zip(cams, dLs)]
    flips = [oracle.render_backward(sc, cam, ost, d[None], near_threshold=G.MARGIN_X)
             for cam, d in zip(cams, dLs)]
    G.check_grads({k: g.cpu().numpy() for k, g in zip(keys, grads)},
                  G.sum_backward(parts, keys, flips))


# -------------------------------------------------- batching, edge cases ---

def test_batched_equals_single(R, dev):
    wl = scenes.config3(n=4000, n_views=5, with_grad=False)
    sc = wl.scene
    cams = [scenes.Camera(c.R, c.t, c.fx / 8, c.fy / 8, c.cx / 8, c.cy / 8, c.width // 8,
                          c.height // 8) for c in wl.cams]
    st = _settings(sh_degree=3, tile=(16, 8))
    t = G.device_scene(sc, dev)
    many = [x.cpu().numpy() for x in R.forward(*t, cams, st)]
    for v, cam in enumerate(cams):
        one = R.forward(*t, [cam], st)[0].cpu().numpy()
        assert np.array_equal(one, many[v])


def test_backward_overwrite_equals_accumulate_into_zeros(R, dev, cfg1):
    """accumulate=False writes every gradient element (stale values in the
    arrays do not leak through, Gaussians nothing reached get 0) and equals
    accumulating into zeroed arrays; accumulating twice doubles."""
    sc, cam = cfg1.scene, cfg1.cams[0]
    st = _settings(act="softplus", tile=(8, 8))
    t = G.device_scene(sc, dev)
    rng = np.random.default_rng(17)
    dL = torch.from_numpy(rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)).to(dev)
    R.forward(*t, [cam], st)
    acc = [torch.zeros_like(x) for x in t]
    R.backward([dL], *acc)
    over = [torch.full_like(x, 7.0) for x in t]
    R.backward([dL], *over, accumulate=False)
    twice = [x.clone() for x in acc]
    R.backward([dL], *twice)
    torch.cuda.synchronize()
    for a, o, w in zip(acc, over, twice):
        a, o, w = a.cpu().numpy(), o.cpu().numpy(), w.cpu().numpy()
        scale = np.abs(a).max() + 1e-30
        # record gradients are summed with FP32 atomics: equal up to their order
        assert np.abs(o - a).max() <= 1e-5 * scale
        assert np.abs(w - 2 * a).max() <= 2e-5 * scale
    untouched = np.all(acc[0].cpu().numpy() == 0, axis=1)
    assert np.all(over[0].cpu().numpy()[untouched] == 0)


def test_empty_and_degenerate(R, dev):
    st = _settings(bg=(0.25, 0.5, 0.75))
    cam = scenes.axis_camera(4.0, 7, 5, 60.0)
    z = torch.zeros((0, 3), device=dev)
    img = R.forward(z, torch.zeros((0, 4), device=dev), z, torch.zeros((0,), device=dev),
                    torch.zeros((0, 1, 3), device=dev), [cam], st)[0].cpu().numpy()
    assert np.allclose(img, np.array([0.25, 0.5, 0.75])[:, None, None])
    # everything behind the camera or zero density: background everywhere
    sc = scenes.config1(n=50, width=7, height=5).scene
    means = sc.means.copy()
    means[:, 2] = -10.0
    sc2 = scenes.Scene(means, sc.quats, sc.scales, sc.dens, sc.sh, 0)
    img = R.forward(*G.device_scene(sc2, dev), [cam], st)[0].cpu().numpy()
    assert np.allclose(img, np.array([0.25, 0.5, 0.75])[:, None, None])
    sc3 = scenes.Scene(sc.means, sc.quats, sc.scales, np.zeros_like(sc.dens), sc.sh, 0)
    img = R.forward(*G.device_scene(sc3, dev), [cam], st)[0].cpu().numpy()
    assert np.allclose(img, np.array([0.25, 0.5, 0.75])[:, None, None])
    # 1x1 image
    cam1 = scenes.axis_camera(4.0, 1, 1, 60.0)
    sc4 = scenes.config1(n=200).scene
    img = R.forward(*G.device_scene(sc4, dev), [cam1], _settings())[0].cpu().numpy()
    ref = oracle.render(sc4, cam1, oracle.Settings())
    assert G.ok_mask(ref).all()
    assert np.abs(img - ref["image"]).max() <= G.IMG_TOL


def test_invalid_arguments(R, dev):
    from paper_2412_03378_amd import _lib
    cam = scenes.axis_camera(4.0, 8, 8, 60.0)
    sc = scenes.config1(n=10, width=8, height=8).scene
    t = G.device_scene(sc, dev)
    with pytest.raises(_lib.VgrError) as e:
        R.forward(*t, [cam], _settings(tile=(12, 12)))
    assert e.value.code == _lib.VGR_ERR_INVALID_ARG
    with pytest.raises(_lib.VgrError) as e:
        R.forward(*t, [cam], _settings(sh_degree=5))
    assert e.value.code == _lib.VGR_ERR_INVALID_ARG


# ------------------------------------------------- hard geometry, ragged ---

def _fwd_bwd_check(R, dev, sc, cam, st, seed):
    """Forward image and backward gradients of one view against the oracle
    (flagged pixels get a zero upstream gradient)."""
    ost = _oset(st)
    ref = oracle.render(sc, cam, ost)
    t = G.device_scene(sc, dev)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    G.check_image(img, ref)
    G.check_emission(R)
    rng = np.random.default_rng(seed)
    dL = G.upstream(rng, ref, 3)
    gref = oracle.render_backward(sc, cam, ost, dL)
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(dL.astype(np.float32)).to(dev)], *grads)
    torch.cuda.synchronize()
    G.check_grads({k: g.cpu().numpy() for k, g in zip(G.GRAD_KEYS, grads)},
                  G.sum_backward([gref], G.GRAD_KEYS))
    return img, ref


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_gaussians_across_the_camera_plane(R, dev, tile):
    """Means in front of the near plane whose bound ellipsoid reaches behind
    the camera (the whole screen is their box; the full-line integral counts
    the part behind the camera), next to means just behind the near plane
    (culled), in front of a field of ordinary Gaussians."""
    rng = np.random.default_rng(21)
    cam = scenes.axis_camera(4.0, 40, 30, 60.0)
    means = [[0.05, -0.02, -3.5], [-0.3, 0.2, -3.7], [0.2, 0.1, -3.79], [0.0, 0.0, -3.81]]
    scales = [[0.4, 0.3, 0.5], [0.2, 0.6, 0.3], [0.05, 0.06, 0.045], [0.3, 0.3, 0.3]]
    dens = [0.3, 0.5, 2.0, 1.0]
    n_field = 300
    means += list(np.c_[rng.uniform(-1, 1, (n_field, 2)), rng.uniform(-1, 1, n_field)])
    scales += list(np.exp(rng.uniform(np.log(0.02), np.log(0.15), (n_field, 3))))
    dens += list(np.exp(rng.uniform(np.log(0.2), np.log(5), n_field)))
    quats = rng.standard_normal((len(means), 4))
    sc = H.scene(means, scales, dens, quats=quats, rgb=rng.uniform(0, 1, (len(means), 3)))
    st = _settings(act="softplus", tile=tile, bg=(0.1, 0.2, 0.3))
    _fwd_bwd_check(R, dev, sc, cam, st, seed=22)


@pytest.mark.parametrize("tile", [(8, 8), (32, 8)])
def test_extreme_anisotropy(R, dev, tile):
    """Needles and disks with axis ratios up to 1e4: the 2x2 bound form is too
    ill-conditioned to keep (no pixel pre-test, no tile culling), alongside
    moderately anisotropic ones."""
    rng = np.random.default_rng(31)
    cam = scenes.axis_camera(4.0, 48, 40, 50.0)
    n = 120
    means = np.c_[rng.uniform(-0.8, 0.8, (n, 2)), rng.uniform(-0.5, 0.5, n)]
    ratio = np.exp(rng.uniform(0, np.log(1e4), n))
    big = np.exp(rng.uniform(np.log(0.05), np.log(0.4), n))
    kind = rng.integers(0, 3, n)
    scales = np.stack([big, big / np.where(kind == 0, ratio, 1.0),
                       big / np.where(kind >= 1, ratio, 1.0)], 1)
    dens = np.exp(rng.uniform(np.log(0.5), np.log(30), n))
    sc = H.scene(means, scales, dens, quats=rng.standard_normal((n, 4)),
                 rgb=rng.uniform(0, 1, (n, 3)))
    st = _settings(tile=tile)
    _fwd_bwd_check(R, dev, sc, cam, st, seed=32)


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8), (16, 16)])
def test_ragged_image_all_tiles(R, dev, cfg1, tile):
    """An image of 37x23 pixels (a partial tile column and row in every tile
    shape), forward and backward against the oracle."""
    sc = cfg1.scene
    cam = scenes.axis_camera(4.0, 37, 23, 60.0)
    st = _settings(act="softplus", tile=tile)
    _fwd_bwd_check(R, dev, sc, cam, st, seed=41)


def test_isotropic_gaussian_has_zero_rotation_gradient(R, dev):
    """An isotropic Gaussian is rotation invariant, so its quaternion gradient
    is exactly zero: the kernels return 0 (the body-frame rotation gradient has
    the factor s_i/s_j - s_j/s_i), and the FP64 oracle returns rounding noise
    far below its scale gradient.  The relative tolerance is not used here
    because both the reference and its per-pixel contributions are noise."""
    rng = np.random.default_rng(51)
    cam = scenes.axis_camera(4.0, 32, 24, 60.0)
    n = 40
    means = np.c_[rng.uniform(-0.6, 0.6, (n, 2)), rng.uniform(-0.5, 0.5, n)]
    s_iso = np.exp(rng.uniform(np.log(0.03), np.log(0.2), n))
    sc = H.scene(means, np.c_[s_iso, s_iso, s_iso], np.exp(rng.uniform(0, np.log(20), n)),
                 quats=rng.standard_normal((n, 4)), rgb=rng.uniform(0, 1, (n, 3)))
    st = _settings(act="softplus", tile=(8, 8))
    ost = _oset(st)
    ref = oracle.render(sc, cam, ost)
    dL = G.upstream(rng, ref, 3)
    gref = oracle.render_backward(sc, cam, ost, dL)
    t = G.device_scene(sc, dev)
    R.forward(*t, [cam], st)
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.from_numpy(dL.astype(np.float32)).to(dev)], *grads)
    torch.cuda.synchronize()
    assert np.all(grads[1].cpu().numpy() == 0.0)
    scale_mag = np.abs(gref["scales"]).max()
    assert scale_mag > 0
    assert np.abs(gref["quats"]).max() <= 1e-9 * scale_mag


def test_emission_of_long_row_lists(R, dev):
    """Large Gaussians on a tall image: every block of 64 depth-sorted
    Gaussians lists far more than 1024 candidate tile rows, so the emission
    walks its rows in several chunks; images and gradients against the
    oracle."""
    rng = np.random.default_rng(61)
    n = 150
    cam = scenes.Camera(np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 4.0], np.float32),
                        300.0, 300.0, 8.0, 1200.0, 16, 2400, 0.2)
    means = np.c_[rng.uniform(-0.3, 0.3, (n, 2)), rng.uniform(-1.0, 1.0, n)]
    scales = np.exp(rng.uniform(np.log(0.8), np.log(2.5), (n, 3)))
    dens = np.exp(rng.uniform(np.log(0.02), np.log(0.2), n))
    sc = H.scene(means, scales, dens, quats=rng.standard_normal((n, 4)),
                 rgb=rng.uniform(0, 1, (n, 3)))
    st = _settings(act="softplus", tile=(8, 8))
    img, ref = _fwd_bwd_check(R, dev, sc, cam, st, seed=62)
    stats = R.stats()
    # the lists really are long: about one instance per Gaussian and tile row
    assert stats["instances"] > 64 * 1024


def test_workgroup_timing_and_pair_counts(R, dev, cfg1):
    """Workgroup timing (production kernels) yields a finite per-CU load
    balance >= 1 without changing the image; pair counting reports blended
    pairs equal in forward and backward (the backward replays exactly the
    forward's blends) and no backward pre-tests."""
    sc, cam = cfg1.scene, cfg1.cams[0]
    st = _settings(tile=(8, 8))
    t = G.device_scene(sc, dev)
    ref = R.forward(*t, [cam], st)[0].cpu().numpy()
    R.set_counting(False, wg_timing=True)
    img = R.forward(*t, [cam], st)[0].cpu().numpy()
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.ones((3, cam.height, cam.width), device=dev)], *grads)
    s = R.stats()
    R.set_counting(False)
    assert np.array_equal(img, ref)
    assert 1.0 <= s["load_balance_fwd"] < 100.0 and 1.0 <= s["load_balance_bwd"] < 100.0
    R.set_counting(True)
    R.forward(*t, [cam], st)
    R.backward([torch.ones((3, cam.height, cam.width), device=dev)], *grads)
    s = R.stats()
    R.set_counting(False)
    assert s["pairs_blended"] > 0 and s["pairs_blended"] == s["bwd_pairs_blended"]
    assert s["bwd_pairs_tested"] == 0
    assert s["pairs_full"] >= s["pairs_blended"] and s["pairs_tested"] >= s["pairs_full"]


@pytest.mark.parametrize("act", ["softplus", "clamp"])
def test_backward_quarters_with_uneven_lists(R, dev, act):
    """8x8 tiles, where each 4x4 quarter of a tile walks its own Gaussians in
    the backward: sub-pixel Gaussians (one quarter each, so the quarters'
    lists differ in length and content) over a few that span whole tiles,
    some tiles left with one busy quarter; image and gradients against the
    oracle, then the walk's counters: every wave step carries one to four
    (Gaussian, quarter) visits."""
    rng = np.random.default_rng(51)
    cam = scenes.axis_camera(4.0, 64, 48, 50.0)
    n_small, n_big = 500, 12
    means = np.r_[np.c_[rng.uniform(-0.9, 0.9, (n_small, 2)), rng.uniform(-0.5, 0.5, n_small)],
                  np.c_[rng.uniform(-0.5, 0.5, (n_big, 2)), rng.uniform(0.3, 0.6, n_big)]]
    # the left third of the frame holds only the small ones
    means[:n_small, 0] = np.where(rng.random(n_small) < 0.4, -0.85 + 0.3 * rng.random(n_small),
                                  means[:n_small, 0])
    scales = np.r_[np.exp(rng.uniform(np.log(0.004), np.log(0.012), (n_small, 3))),
                   np.exp(rng.uniform(np.log(0.15), np.log(0.35), (n_big, 3)))]
    dens = np.r_[np.exp(rng.uniform(np.log(5.0), np.log(60.0), n_small)),
                 np.exp(rng.uniform(np.log(0.3), np.log(2.0), n_big))]
    sc = H.scene(means, scales, dens, quats=rng.standard_normal((n_small + n_big, 4)),
                 rgb=rng.uniform(0, 1, (n_small + n_big, 3)))
    st = _settings(act=act, tile=(8, 8), bg=(0.2, 0.1, 0.3))
    _fwd_bwd_check(R, dev, sc, cam, st, seed=52)
    t = G.device_scene(sc, dev)
    R.set_counting(True)
    R.forward(*t, [cam], st)
    grads = [torch.zeros_like(x) for x in t]
    R.backward([torch.ones((3, cam.height, cam.width), device=dev)], *grads)
    s = R.stats()
    R.set_counting(False)
    steps, visits = s["bwd_visits"], s["bwd_visits_full"]
    print(f"backward steps {steps}, (Gaussian, quarter) visits {visits}, "
          f"pairs {s['bwd_pairs_full']}")
    assert 0 < steps <= visits <= 4 * steps
    assert s["bwd_pairs_full"] <= 16 * visits
    assert s["pairs_blended"] == s["bwd_pairs_blended"]
