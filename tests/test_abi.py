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
    # alpha_model, near_segment, tile_resort
    assert ctypes.sizeof(_lib.vgr_settings) == 4 * (2 + 4 + 3 + 1 + 2 + 4)


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
