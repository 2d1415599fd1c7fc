"""The allocation-free sort entry point (vgr_sort_pairs_static) against the
allocating one (vgr_sort_pairs), through the C ABI: identical keys and values
(integer work, bit for bit) on two calls in a row, the second smaller, and
sizes past the static scratch rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pairs(n, bits, seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
    v = rng.permutation(n).astype(np.uint32)
    return k, v


def test_static_sort_matches_allocating_sort():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2412_03378_amd import Renderer, _lib as L
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    lib = r._lib
    # two calls in a row, the second smaller (its scratch holds the first
    # call's data); then the largest size the scratch holds
    for n, bits, seed in ((300001, 20, 1), (4097, 13, 2), (L.VGR_STATIC_SORT_MAX, 32, 3)):
        k, v = _pairs(n, bits, seed)
        ka = torch.from_numpy(k.view(np.int32)).to(dev)
        va = torch.from_numpy(v.view(np.int32)).to(dev)
        kb, vb = ka.clone(), va.clone()
        print(f"static sort n={n} bits={bits}", flush=True)
        rc = lib.vgr_sort_pairs_static(r._h, C.c_void_p(kb.data_ptr()), C.c_void_p(vb.data_ptr()),
                                       n, bits)
        L.check(rc, r._h)
        r.sort_pairs(ka, va, bits)
        torch.cuda.synchronize()
        assert np.array_equal(kb.cpu().numpy(), ka.cpu().numpy())
        assert np.array_equal(vb.cpu().numpy(), va.cpu().numpy())
        order = np.argsort(k, kind="stable")
        assert np.array_equal(kb.cpu().numpy().view(np.uint32), k[order])
    big = torch.zeros(L.VGR_STATIC_SORT_MAX + 1, dtype=torch.int32, device=dev)
    rc = lib.vgr_sort_pairs_static(r._h, C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()),
                                   big.numel(), 8)
    assert rc == L.VGR_ERR_INVALID_ARG
    assert b"static scratch" in lib.vgr_last_error(r._h)
    r.close()
