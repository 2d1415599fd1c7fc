"""The C ABI library loads and exports every function include/vgr.h declares
(no device calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "vgr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vgr_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    from paper_2412_03378_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2412_03378_amd.build import build
        build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(_lib.EXPORTED) == names


def test_header_structs_match_binding():
    from paper_2412_03378_amd import _lib
    assert ctypes.sizeof(_lib.vgr_camera) == 4 * (9 + 3 + 4 + 2 + 1 + 1)
    assert ctypes.sizeof(_lib.vgr_settings) == 4 * (2 + 4 + 3 + 1 + 2 + 2)


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2412_03378_amd import _lib
    import pytest
    with pytest.raises(ImportError):
        _lib._lib, saved = None, _lib._lib
        try:
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = saved
