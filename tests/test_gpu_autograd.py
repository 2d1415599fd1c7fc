"""The torch.autograd.Function binding: loss.backward() through render()
gives the gradients of the explicit C ABI backward (same kernels)."""
import numpy as np
import pytest

import gpu_helpers as G
from paper_2412_03378_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("mode,opt", [("color", {}), ("xray", {}), ("color", {"density": "theta"}),
                                      ("color", {"alpha_model": "splat"}),
                                      ("xray", {"near_segment": True}),
                                      ("color", {"tile_resort": True}),
                                      ("color", {"kernel": "epanechnikov"}),
                                      ("xray", {"kernel": "epanechnikov"})])
def test_autograd_matches_explicit_backward(mode, opt):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2412_03378_amd import Renderer, Settings, render
    dev = torch.device("cuda", 0)
    wl = scenes.config1(n=400, width=40, height=32)
    if opt.get("density") == "theta":
        wl.scene = scenes.with_theta(wl.scene, seed=7)
    if opt.get("alpha_model") == "splat":
        wl.scene = scenes.with_opacity(wl.scene, seed=8)
    cams = [wl.cams[0], scenes.axis_camera(3.5, 24, 20, 50.0)]
    st = Settings(mode=mode, tile=(8, 8), **opt)
    t = [x.clone().requires_grad_(True) if x is not None else None
         for x in G.device_scene(wl.scene, dev)]
    if mode == "xray":
        t[4] = None
    imgs = render(*t, cams, st)
    rng = np.random.default_rng(3)
    w = [torch.from_numpy(rng.standard_normal(tuple(i.shape)).astype(np.float32)).to(dev)
         for i in imgs]
    loss = sum((i * wi).sum() for i, wi in zip(imgs, w))
    loss.backward()
    r = Renderer(0)
    base = [x.detach() if x is not None else None for x in t]
    r.forward(*base, cams, st)
    grads = [torch.zeros_like(x) if x is not None else None for x in base]
    r.backward(w, *grads)
    torch.cuda.synchronize()
    for a, b in zip(t, grads):
        if a is None:
            continue
        assert np.allclose(a.grad.cpu().numpy(), b.cpu().numpy(), rtol=1e-4,
                           atol=1e-6 * float(b.abs().max()) + 1e-12)


def test_render_reuses_pooled_contexts_and_refuses_foreign_backward():
    """render() without a renderer takes a pooled context: two pending nodes
    hold two contexts, and after their backwards the next render reuses one
    of them.  A node whose explicit renderer has run another forward since
    refuses to differentiate (the library keeps only the last forward)."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2412_03378_amd import Renderer, Settings, render
    from paper_2412_03378_amd import renderer as RM
    dev = torch.device("cuda", 0)
    wl = scenes.config1(n=200, width=24, height=16)
    st = Settings(tile=(8, 8))
    t = [x.clone().requires_grad_(True) for x in G.device_scene(wl.scene, dev)]
    a = render(*t, wl.cams, st)
    b = render(*t, wl.cams, st)
    ra, rb = a[0].grad_fn.renderer, b[0].grad_fn.renderer
    assert ra is not rb
    (a[0].sum() + b[0].sum()).backward()
    c = render(*t, wl.cams, st)
    assert c[0].grad_fn.renderer in (ra, rb)
    assert len(RM._POOL[0]) >= 2
    c[0].sum().backward()
    # one explicit context, two forwards, backward of the first: refused
    r = Renderer(0)
    first = render(*t, wl.cams, st, renderer=r)
    render(*t, wl.cams, st, renderer=r)
    with pytest.raises(RuntimeError, match="another forward"):
        first[0].sum().backward()
    r.close()
