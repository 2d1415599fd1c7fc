"""The oracle's algorithm evaluated in FP32: the same C source compiled with
every ``double`` read as ``float`` (tgmath.h for the math functions,
single-precision constants).  It measures what FP32 rounding does to the
gradients of this computation (tests/test_fp32_error_model.py) and is never a
reference for anything."""
import ctypes as C
import os
import subprocess

import numpy as np

import oracle


class _SettingsF(C.Structure):
    _fields_ = [("mode", C.c_int32), ("sh_degree", C.c_int32), ("act", C.c_int32),
                ("density", C.c_int32), ("alpha_model", C.c_int32), ("near_segment", C.c_int32),
                ("tile_resort", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("kernel", C.c_int32), ("pixel_window", C.c_int32), ("pad3", C.c_int32),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("T_min", C.c_float), ("x_min_xray", C.c_float), ("bg", C.c_float * 3),
                ("near_threshold", C.c_float)]


def build(out_dir):
    """Compile the FP32 variant into out_dir; returns the loaded library."""
    src = open(oracle._SRC).read().split("\n")
    # after the system headers, before the first definition
    first = next(i for i, l in enumerate(src) if l.startswith("#define ORC_"))
    src.insert(first, "#include <tgmath.h>\n#undef I\n#undef complex\n#define double float")
    c_path = os.path.join(out_dir, "vgr_oracle_f32.c")
    so_path = os.path.join(out_dir, "liboracle_f32.so")
    with open(c_path, "w") as f:
        f.write("\n".join(src))
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fsingle-precision-constant", "-w", "-o", so_path, c_path, "-lm"], check=True)
    lib = C.CDLL(so_path)
    fp = C.POINTER(C.c_float)
    ip = C.POINTER(C.c_int32)
    lib.orc_render_backward.argtypes = [C.c_int64, fp, fp, fp, fp, fp, C.POINTER(oracle._Cam),
                                        C.POINTER(_SettingsF), C.c_int64, ip, fp] + [fp] * 15
    lib.orc_render.argtypes = [C.c_int64, fp, fp, fp, fp, fp, C.POINTER(oracle._Cam),
                               C.POINTER(_SettingsF), C.c_int64, ip, fp, fp,
                               C.POINTER(C.c_int64), ip, fp, fp]
    return lib


def _settings(st, sh_degree):
    d = oracle._settings(st, sh_degree)
    s = _SettingsF()
    for name, _ in _SettingsF._fields_:
        if name == "bg":
            s.bg[:] = [float(v) for v in d.bg]
        else:
            setattr(s, name, getattr(d, name))
    return s


def render_backward(lib, scene, cam, st, dL):
    """FP32 gradients of sum(dL * image) over the whole image (dict of float64
    copies of the float32 results)."""
    pix = oracle.all_pixels(cam)
    P = pix.shape[0]
    nch = 1 if st.mode == "xray" else 3
    g = np.ascontiguousarray(np.asarray(dL, np.float32).reshape(nch, P).T)
    means, quats, scales, dens, sh = oracle._scene_arrays(scene, st.mode)
    n = means.shape[0]
    nb = (scene.sh_degree + 1) ** 2
    shapes = dict(means=(n, 3), quats=(n, 4), scales=(n, 3), dens=(n,), sh=(n, nb, 3))
    keys = tuple(shapes)
    out = {k: [np.zeros(s, np.float32) for _ in range(3)] for k, s in shapes.items()}
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))
    cam_s, set_s = oracle._cam(cam), _settings(st, scene.sh_degree)
    rc = lib.orc_render_backward(int(n), ptr(means), ptr(quats), ptr(scales), ptr(dens), ptr(sh),
                                 C.byref(cam_s), C.byref(set_s), P,
                                 pix.ctypes.data_as(C.POINTER(C.c_int32)), ptr(g),
                                 *[ptr(out[k][0]) for k in keys], *[ptr(out[k][1]) for k in keys],
                                 *[ptr(out[k][2]) for k in keys])
    if rc:
        raise RuntimeError(f"FP32 orc_render_backward failed ({rc})")
    return {k: out[k][0].astype(np.float64) for k in keys}


def render(lib, scene, cam, st):
    """FP32 image (C, H, W) as float64."""
    pix = oracle.all_pixels(cam)
    P = pix.shape[0]
    nch = 1 if st.mode == "xray" else 3
    means, quats, scales, dens, sh = oracle._scene_arrays(scene, st.mode)
    out = np.zeros((P, nch), np.float32)
    T = np.zeros(P, np.float32)
    last = np.zeros(P, np.int64)
    nbl = np.zeros(P, np.int32)
    marg = np.zeros((P, 3), np.float32)
    untr = np.zeros(P, np.float32)
    fp = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))
    cam_s, set_s = oracle._cam(cam), _settings(st, scene.sh_degree)
    rc = lib.orc_render(int(means.shape[0]), fp(means), fp(quats), fp(scales), fp(dens), fp(sh),
                        C.byref(cam_s), C.byref(set_s), P, pix.ctypes.data_as(C.POINTER(C.c_int32)),
                        fp(out), fp(T), last.ctypes.data_as(C.POINTER(C.c_int64)),
                        nbl.ctypes.data_as(C.POINTER(C.c_int32)), fp(marg), fp(untr))
    if rc:
        raise RuntimeError(f"FP32 orc_render failed ({rc})")
    return out.T.astype(np.float64).reshape(nch, int(cam.height), int(cam.width))
