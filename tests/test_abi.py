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
    # mode, sh_degree; 4 thresholds; bg; act; tile_w, tile_h; density,
    # alpha_model, near_segment, tile_resort, kernel, batch, pixel_window
    assert ctypes.sizeof(_lib.vgr_settings) == 4 * (2 + 4 + 3 + 1 + 2 + 7)


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2412_03378_amd import _lib
    import pytest
    with pytest.raises(ImportError):
        _lib._lib, saved = None, _lib._lib
        try:
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = saved


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of the public structs have the C compiler's sizes and
    field offsets for include/vgr.h."""
    import subprocess
    from paper_2412_03378_amd import _lib
    src = tmp_path / "layout.c"
    fields = {name: [f for f, _ in getattr(_lib, name)._fields_]
              for name in ("vgr_camera", "vgr_settings", "vgr_stats")}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vgr.h"', "int main(void) {"]
    for name, fs in fields.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in fs:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = dict(zip(out[0::2], (int(x) for x in out[1::2])))
    for name, fs in fields.items():
        st = getattr(_lib, name)
        assert got[name] == ctypes.sizeof(st), name
        for f in fs:
            assert got[f"{name}.{f}"] == getattr(st, f).offset, (name, f)


def test_default_settings_are_the_documented_ones():
    from paper_2412_03378_amd import _lib
    lib = _lib.load()
    s = _lib.vgr_settings()
    lib.vgr_default_settings(ctypes.byref(s))
    assert s.mode == _lib.VGR_MODE_COLOR and s.sh_degree == 0
    assert abs(s.alpha_min - 1 / 255) < 1e-9 and abs(s.alpha_max - 0.99) < 1e-7
    assert abs(s.T_min - 1e-4) < 1e-11 and abs(s.x_min_xray - 1e-6) < 1e-13
    assert list(s.bg) == [0.0, 0.0, 0.0] and s.act == _lib.VGR_ACT_CLAMP0
    assert (s.tile_w, s.tile_h) == (0, 0)
    assert s.density == _lib.VGR_DENSITY_KAPPA and s.alpha_model == _lib.VGR_ALPHA_VOLUMETRIC
    assert s.near_segment == 0 and s.tile_resort == 0


def test_null_context_calls_fail_cleanly():
    """Every entry point given a NULL context returns VGR_ERR_INVALID_ARG
    (nothing is thrown, nothing touches a device)."""
    from paper_2412_03378_amd import _lib
    lib = _lib.load()
    E = _lib.VGR_ERR_INVALID_ARG
    assert lib.vgr_set_stream(None, None) == E
    assert lib.vgr_set_counting(None, 1) == E
    assert lib.vgr_set_timing(None, 1) == E
    assert lib.vgr_set_densify_stats(None, None, None, 0) == E
    assert lib.vgr_graph_launch(None) == E
    assert lib.vgr_render_backward(None, None, None, None, None, None, None, 0) == E
    assert lib.vgr_get_stats(None, None) == E
    assert isinstance(lib.vgr_last_error(None), bytes)
    lib.vgr_destroy(None)


def test_create_without_a_device_returns_an_error():
    import pytest
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2412_03378_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.vgr_create(ctypes.byref(h), 0)
    assert rc < 0 and not h.value
