"""hipGraph capture of a whole forward+backward step, and the autotuner.

A captured step is replayed several times with ordinary eager work and
synchronisations between replays; every replay must equal the eager result
bit for bit.  Capacity overflow is forced from the host (the scene grows after
capture) and must be reported, not silently ignored.
"""
import numpy as np
import pytest

import gpu_helpers as G
from paper_2412_03378_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _setup(dev, n=3000, views=3, seed=8):
    from paper_2412_03378_amd import Settings
    wl = scenes.config3(n=n, n_views=8, seed=seed, with_grad=False)
    cams = [scenes.Camera(c.R, c.t, c.fx / 6, c.fy / 6, c.cx / 6, c.cy / 6, c.width // 6,
                          c.height // 6) for c in wl.cams[:views]]
    params = list(G.device_scene(wl.scene, dev))
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in cams]
    rng = np.random.default_rng(seed)
    dL = [torch.from_numpy(rng.standard_normal((3, c.height, c.width)).astype(np.float32)).to(dev)
          for c in cams]
    grads = [torch.zeros_like(p) for p in params]
    return Settings(sh_degree=3, tile=(16, 8)), cams, params, outs, dL, grads


def _eager(dev, st, cams, params, dL):
    from paper_2412_03378_amd import Renderer
    r = Renderer(0)
    imgs = [x.clone() for x in r.forward(*params, cams, st)]
    grads = [torch.zeros_like(p) for p in params]
    r.backward(dL, *grads)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in imgs], [g.cpu().numpy() for g in grads]


def test_graph_replays_equal_eager(dev):
    from paper_2412_03378_amd import Renderer
    st, cams, params, outs, dL, grads = _setup(dev)
    ref_img, ref_g = _eager(dev, st, cams, params, dL)
    r = Renderer(0)
    r.graph_capture(params, cams, st, outs, dL, grads, capacity_factor=1.25, zero_grads=True)
    for rep in range(4):
        for o in outs:
            o.fill_(-1.0)
        r.graph_launch()
        r.graph_check()
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        for a, b in zip(outs, ref_img):
            assert np.array_equal(a.cpu().numpy(), b), f"replay {rep}"
        for a, b in zip(grads, ref_g):
            # gradient sums use FP32 atomics: equal up to the order of additions
            assert np.allclose(a.cpu().numpy(), b, rtol=1e-4, atol=1e-6 * np.abs(b).max()), rep


def test_graph_overflow_is_reported(dev):
    from paper_2412_03378_amd import Renderer, _lib
    st, cams, params, outs, dL, grads = _setup(dev, seed=9)
    r = Renderer(0)
    r.graph_capture(params, cams, st, outs, dL, grads, capacity_factor=1.0)
    r.graph_launch()
    r.graph_check()
    params[2].mul_(3.0)     # bigger Gaussians cover more tiles than captured
    r.graph_launch()
    with pytest.raises(_lib.VgrError) as e:
        r.graph_check()
    assert e.value.code == _lib.VGR_ERR_CAPACITY
    # a new capture fits the grown scene and matches the eager result again
    ref_img, _ = _eager(dev, st, cams, params, dL)
    r.graph_capture(params, cams, st, outs, dL, grads, capacity_factor=1.25)
    r.graph_launch()
    r.graph_check()
    for a, b in zip(outs, ref_img):
        assert np.array_equal(a.cpu().numpy(), b)


def test_autotune_picks_a_valid_shape_and_caches_it_per_workload(dev):
    """The tuner times every (tile, records per batch) candidate; calls of the
    same workload class that leave the shape to the library use its choice
    (bitwise the explicit result); the choice exports as text and another
    context that imports it makes the same choice; malformed text is
    rejected whole."""
    from paper_2412_03378_amd import Renderer, Settings, _lib
    st, cams, params, outs, dL, grads = _setup(dev, seed=10)
    r = Renderer(0)
    best, batch, ms = r.autotune(params, cams, st, outs, dL, grads, iters=2)
    assert best in [(8, 8), (16, 8), (16, 16), (32, 8)] and batch in (32, 64)
    assert len(ms) == _lib.VGR_TUNE_CANDIDATES and all(m > 0 for m in ms)
    auto = [x.cpu().numpy() for x in r.forward(*params, cams, Settings(sh_degree=3))]
    explicit = [x.cpu().numpy() for x in r.forward(*params, cams,
                                                   Settings(sh_degree=3, tile=best, batch=batch))]
    for a, b in zip(auto, explicit):
        assert np.array_equal(a, b)
    assert r.stats()["tile_w"] == best[0]
    text = r.tuning_text()
    fields = text.strip().split()
    assert len(fields) == 11 and (int(fields[7]), int(fields[8])) == best and int(fields[9]) == batch
    r2 = Renderer(0)
    r2.load_tuning(text)
    r2.forward(*params, cams, Settings(sh_degree=3))
    assert (r2.stats()["tile_w"], r2.stats()["tile_h"]) == best
    # another workload class (X-ray) is not affected by the colour entry
    with pytest.raises(_lib.VgrError) as e:
        r2.load_tuning("1 2 3\n")
    assert e.value.code == _lib.VGR_ERR_INVALID_ARG
    with pytest.raises(_lib.VgrError):
        r2.load_tuning(text.replace(f" {batch} ", " 48 ", 1))
    r.close()
    r2.close()


def test_multi_call_graph_replays_equal_eager(dev):
    """Three forward + backward calls of 2, 1 and 2 views captured in one
    graph: every replay gives the eager calls' images exactly and their summed
    gradients up to the order of the FP32 atomics."""
    from paper_2412_03378_amd import Renderer, Settings
    wl = scenes.config3(n=3000, n_views=5, seed=12, with_grad=False)
    cams = [scenes.Camera(c.R, c.t, c.fx / 6, c.fy / 6, c.cx / 6, c.cy / 6, c.width // 6,
                          c.height // 6) for c in wl.cams]
    params = list(G.device_scene(wl.scene, dev))
    rng = np.random.default_rng(12)
    dL = [torch.from_numpy(rng.standard_normal((3, c.height, c.width)).astype(np.float32)).to(dev)
          for c in cams]
    st = Settings(sh_degree=3, tile=(16, 8))
    split = [2, 1, 2]
    e = Renderer(0)
    ref_img, ref_g = [], [torch.zeros_like(p) for p in params]
    v0 = 0
    for k, nv in enumerate(split):
        imgs = e.forward(*params, cams[v0:v0 + nv], st)
        ref_img += [x.cpu().numpy() for x in imgs]
        e.backward(dL[v0:v0 + nv], *ref_g, accumulate=k > 0)
        v0 += nv
    torch.cuda.synchronize()
    ref_g = [g.cpu().numpy() for g in ref_g]
    r = Renderer(0)
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in cams]
    grads = [torch.full_like(p, 3.0) for p in params]
    r.graph_capture_calls(params, cams, split, st, outs, dL, grads, capacity_factor=1.25,
                          zero_grads=True)
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        r.graph_launch()
        r.graph_check()
        junk = torch.randn(1 << 18, device=dev).sum()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        for a, b in zip(outs, ref_img):
            assert np.array_equal(a.cpu().numpy(), b), rep
        for a, b in zip(grads, ref_g):
            assert np.allclose(a.cpu().numpy(), b, rtol=1e-4, atol=1e-6 * np.abs(b).max()), rep
    r.close()
    e.close()


@pytest.mark.parametrize("opt", [{"alpha_model": "splat"}, {"near_segment": True, "density": "theta"},
                                 {"tile_resort": True}])
def test_graph_replays_with_options(opt):
    """A captured step with the training and comparison options replays to
    the eager step's images and gradients (up to the order of the backward's
    FP32 atomics), replay after replay."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2412_03378_amd import Renderer, Settings
    dev = torch.device("cuda", 0)
    wl = scenes.config1(n=600, width=48, height=40)
    sc = wl.scene
    if opt.get("alpha_model") == "splat":
        sc = scenes.with_opacity(sc, seed=9)
    if opt.get("density") == "theta":
        sc = scenes.with_theta(sc, seed=10)
    cam = scenes.Camera(wl.cams[0].R, wl.cams[0].t, wl.cams[0].fx, wl.cams[0].fy,
                        wl.cams[0].cx, wl.cams[0].cy, 48, 40, znear=3.3)
    st = Settings(act="softplus", tile=(8, 8), **opt)
    t = G.device_scene(sc, dev)
    dL = [torch.from_numpy(np.random.default_rng(11).standard_normal(
        (3, 40, 48)).astype(np.float32)).to(dev)]
    ref = Renderer(0)
    img = ref.forward(*t, [cam], st)[0].clone()
    g_ref = [torch.zeros_like(x) for x in t]
    ref.backward(dL, *g_ref, accumulate=False)
    torch.cuda.synchronize()
    r = Renderer(0)
    outs = [torch.empty((3, 40, 48), device=dev)]
    grads = [torch.zeros_like(x) for x in t]
    r.graph_capture(t, [cam], st, outs, dL, grads)
    for _ in range(3):
        r.graph_launch()
        r.graph_check()
        torch.cuda.synchronize()
        assert torch.equal(outs[0], img)
        for a, b in zip(grads, g_ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.allclose(a, b, rtol=1e-4, atol=1e-5 * float(np.abs(b).max()) + 1e-12)
