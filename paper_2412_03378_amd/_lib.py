"""ctypes declarations of libvgr (include/vgr.h).  Argument marshalling only.

The library is loaded from this package directory; if it has not been built
the import fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvgr.so")

VGR_OK = 0
VGR_ERR_INVALID_ARG = -1
VGR_ERR_HIP = -2
VGR_ERR_OOM = -3
VGR_ERR_CAPACITY = -4
VGR_ERR_NOT_CAPTURED = -5
VGR_ERR_NO_FORWARD = -6
VGR_STATIC_SORT_MAX = 1 << 20   # include/vgr.h
VGR_TUNE_CANDIDATES = 8
VGR_MAX_GRAPH_CALLS = 16

VGR_MODE_COLOR = 0
VGR_MODE_XRAY = 1
VGR_ACT_CLAMP0 = 0
VGR_ACT_SOFTPLUS10 = 1
VGR_DENSITY_KAPPA = 0
VGR_DENSITY_THETA = 1
VGR_ALPHA_VOLUMETRIC = 0
VGR_ALPHA_SPLAT = 1
VGR_KERNEL_GAUSSIAN = 0
VGR_KERNEL_EPANECHNIKOV = 1
VGR_MAX_PIXEL_WINDOW = 32


class vgr_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("znear", C.c_float), ("reserved", C.c_int32)]


class vgr_settings(C.Structure):
    _fields_ = [("mode", C.c_int32), ("sh_degree", C.c_int32), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("T_min", C.c_float), ("x_min_xray", C.c_float),
                ("bg", C.c_float * 3), ("act", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("density", C.c_int32), ("alpha_model", C.c_int32),
                ("near_segment", C.c_int32), ("tile_resort", C.c_int32), ("kernel", C.c_int32),
                ("batch", C.c_int32), ("pixel_window", C.c_int32)]


class vgr_stats(C.Structure):
    _fields_ = [("instances", C.c_int64), ("capacity", C.c_int64), ("visible", C.c_int64),
                ("pairs_tested", C.c_int64), ("pairs_full", C.c_int64),
                ("pairs_blended", C.c_int64), ("visits", C.c_int64),
                ("visits_full", C.c_int64), ("bwd_pairs_tested", C.c_int64),
                ("bwd_pairs_full", C.c_int64), ("bwd_pairs_blended", C.c_int64),
                ("bwd_visits", C.c_int64), ("bwd_visits_full", C.c_int64),
                ("overflow", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("n_views", C.c_int32),
                ("load_balance_fwd", C.c_double), ("load_balance_bwd", C.c_double),
                ("emit_mismatch", C.c_int32), ("_pad", C.c_int32)]


class VgrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vgr error {code}: {msg}")
        self.code = code


_lib = None

_SIGNATURES = {
    "vgr_default_settings": (None, [C.POINTER(vgr_settings)]),
    "vgr_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "vgr_destroy": (None, [C.c_void_p]),
    "vgr_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vgr_last_error": (C.c_char_p, [C.c_void_p]),
    "vgr_render_forward": (C.c_int, [C.c_void_p, C.POINTER(vgr_settings), C.c_int64,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int32, C.POINTER(vgr_camera), C.POINTER(C.c_void_p)]),
    "vgr_render_backward": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "vgr_get_aux": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "vgr_get_stats": (C.c_int, [C.c_void_p, C.POINTER(vgr_stats)]),
    "vgr_set_counting": (C.c_int, [C.c_void_p, C.c_int]),
    "vgr_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "vgr_set_densify_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "vgr_get_timing": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_char_p),
                                 C.POINTER(C.c_float), C.POINTER(C.c_int32)]),
    "vgr_sort_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "vgr_sort_pairs_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_int32]),
    "vgr_graph_capture": (C.c_int, [C.c_void_p, C.POINTER(vgr_settings), C.c_int64, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.POINTER(vgr_camera), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_float, C.c_int32]),
    "vgr_graph_capture_calls": (C.c_int, [C.c_void_p, C.POINTER(vgr_settings), C.c_int64,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(vgr_camera), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                          C.c_int32]),
    "vgr_graph_launch": (C.c_int, [C.c_void_p]),
    "vgr_graph_check": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "vgr_autotune": (C.c_int, [C.c_void_p, C.POINTER(vgr_settings), C.c_int64, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                               C.POINTER(vgr_camera), C.POINTER(C.c_void_p),
                               C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "vgr_tune_export": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)]),
    "vgr_tune_import": (C.c_int, [C.c_void_p, C.c_char_p]),
}

EXPORTED = tuple(_SIGNATURES)


def load(path: str = LIB_PATH):
    """Load libvgr.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2412_03378_amd.build.build() first")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, ctx=None):
    if rc != VGR_OK:
        msg = ""
        if ctx is not None and _lib is not None:
            raw = _lib.vgr_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise VgrError(rc, msg)
