"""Python face of libvgr: a context wrapper over PyTorch device tensors and a
``torch.autograd.Function``.  Every step of the rendering runs in the HIP
library; this module only marshals pointers, shapes and the stream.
"""
from __future__ import annotations

import ctypes as C
import threading
import weakref
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _lib as L


@dataclass
class Settings:
    """Rendering rules (see vgr_settings in include/vgr.h)."""
    mode: str = "color"              # "color" | "xray"
    sh_degree: int = 0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    x_min_xray: float = 1e-6
    bg: tuple = (0.0, 0.0, 0.0)
    act: str = "clamp"               # "clamp" | "softplus"
    tile: tuple = (0, 0)             # (0, 0): the context's tuned tile
    density: str = "kappa"           # "kappa" | "theta": what `dens` holds
    alpha_model: str = "volumetric"  # "volumetric" | "splat" (the 3DGS comparison model)
    near_segment: bool = False       # integrate each ray from the near plane on
    tile_resort: bool = False        # per-tile order by the depth of each maximum
    kernel: str = "gaussian"         # "gaussian" | "epanechnikov" (compact primitive)
    batch: int = 0                   # records per rasteriser batch: 32, 64, 0 = tuned
    pixel_window: int = 0            # per-pixel re-sorting window (with tile_resort; 8x8)

    def to_c(self) -> L.vgr_settings:
        s = L.vgr_settings()
        s.mode = L.VGR_MODE_XRAY if self.mode == "xray" else L.VGR_MODE_COLOR
        s.sh_degree = int(self.sh_degree)
        s.alpha_min, s.alpha_max = float(self.alpha_min), float(self.alpha_max)
        s.T_min, s.x_min_xray = float(self.T_min), float(self.x_min_xray)
        s.bg[:] = [float(v) for v in self.bg]
        s.act = L.VGR_ACT_SOFTPLUS10 if self.act == "softplus" else L.VGR_ACT_CLAMP0
        s.tile_w, s.tile_h = int(self.tile[0]), int(self.tile[1])
        s.density = L.VGR_DENSITY_THETA if self.density == "theta" else L.VGR_DENSITY_KAPPA
        s.alpha_model = L.VGR_ALPHA_SPLAT if self.alpha_model == "splat" else L.VGR_ALPHA_VOLUMETRIC
        s.near_segment = 1 if self.near_segment else 0
        s.tile_resort = 1 if self.tile_resort else 0
        s.kernel = L.VGR_KERNEL_EPANECHNIKOV if self.kernel == "epanechnikov" else L.VGR_KERNEL_GAUSSIAN
        s.batch = int(self.batch)
        s.pixel_window = int(self.pixel_window)
        return s

    @staticmethod
    def no_thresholds(mode="color", act="softplus", bg=(0.0, 0.0, 0.0), sh_degree=0,
                      density="kappa", near_segment=False, kernel="gaussian"):
        """Smallest thresholds FP32 allows (for finite-difference checks)."""
        return Settings(mode=mode, sh_degree=sh_degree, alpha_min=1e-30, alpha_max=1 - 2 ** -20,
                        T_min=0.0, x_min_xray=1e-30, bg=bg, act=act, density=density,
                        near_segment=near_segment, kernel=kernel)


def camera_struct(cam) -> L.vgr_camera:
    """Any object with R (3x3), t (3), fx, fy, cx, cy, width, height, znear."""
    c = L.vgr_camera()
    R = [float(v) for v in torch.as_tensor(cam.R, dtype=torch.float32).reshape(9)]
    t = [float(v) for v in torch.as_tensor(cam.t, dtype=torch.float32).reshape(3)]
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def _dev_ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != torch.float32 and t.dtype != torch.int32 and t.dtype != torch.uint32:
        raise ValueError(f"unexpected dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


class Renderer:
    """Owns one vgr context (workspace + the state saved by the last forward)."""

    def __init__(self, device: int = 0):
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.vgr_create(C.byref(h), int(device)))
        self._h = h
        self.device = int(device)
        self.n_views = 0
        self.shapes = []
        self.mode = "color"
        # forwards run so far: an autograd node remembers the number of its
        # own forward and refuses to differentiate another one
        self.generation = 0
        self._owner = None   # weak reference to the autograd node holding this context

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vgr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        L.check(self._lib.vgr_set_stream(self._h, C.c_void_p(s)), self._h)

    def forward(self, means, quats, scales, dens, sh, cams: Sequence, settings: Settings,
                outs: Optional[List[torch.Tensor]] = None) -> List[torch.Tensor]:
        """Render ``cams`` (host camera objects).  Returns one image per view:
        (3, H, W) in colour mode, (H, W) in X-ray mode."""
        self._sync_stream()
        n = int(means.shape[0])
        ncam = len(cams)
        cam_arr = (L.vgr_camera * ncam)(*[camera_struct(c) for c in cams])
        if outs is None:
            outs = []
            for c in cams:
                shape = (int(c.height), int(c.width)) if settings.mode == "xray" else \
                        (3, int(c.height), int(c.width))
                outs.append(torch.empty(shape, dtype=torch.float32, device=means.device))
        out_ptrs = (C.c_void_p * ncam)(*[o.data_ptr() for o in outs])
        st = settings.to_c()
        rc = self._lib.vgr_render_forward(
            self._h, C.byref(st), n, _dev_ptr(means), _dev_ptr(quats), _dev_ptr(scales),
            _dev_ptr(dens), _dev_ptr(sh) if settings.mode != "xray" else None, ncam, cam_arr,
            out_ptrs)
        self.generation += 1
        L.check(rc, self._h)
        self.n_views = ncam
        self.shapes = [tuple(o.shape) for o in outs]
        self.mode = settings.mode
        return outs

    def backward(self, dL: Sequence[torch.Tensor], d_means, d_quats, d_scales, d_dens, d_sh,
                 accumulate: bool = True):
        """Gradients of the last forward: added to the given tensors, or written
        over them (no zeroing needed) when accumulate is False."""
        self._sync_stream()
        dLc = [g.contiguous().float() for g in dL]
        ptrs = (C.c_void_p * len(dLc))(*[g.data_ptr() for g in dLc])
        rc = self._lib.vgr_render_backward(self._h, ptrs, _dev_ptr(d_means), _dev_ptr(d_quats),
                                           _dev_ptr(d_scales), _dev_ptr(d_dens),
                                           _dev_ptr(d_sh), int(bool(accumulate)))
        L.check(rc, self._h)

    def aux(self, view: int, height: int, width: int, device=None):
        """(T_final, last contributor index) of one view of the last forward."""
        self._sync_stream()
        dev = device or torch.device("cuda", self.device)
        T = torch.empty((height, width), dtype=torch.float32, device=dev)
        last = torch.empty((height, width), dtype=torch.int32, device=dev)
        L.check(self._lib.vgr_get_aux(self._h, int(view), _dev_ptr(T), _dev_ptr(last)), self._h)
        return T, last

    def stats(self) -> dict:
        s = L.vgr_stats()
        L.check(self._lib.vgr_get_stats(self._h, C.byref(s)), self._h)
        return {k: getattr(s, k) for k, _ in L.vgr_stats._fields_}

    def set_counting(self, on: bool, wg_timing: bool = False):
        """on: pair counting (instrumented kernels); wg_timing: per-workgroup
        timing of the production rasterisers (load balance in stats())."""
        L.check(self._lib.vgr_set_counting(self._h, int(bool(on)) | (2 if wg_timing else 0)),
                self._h)

    def set_densify_stats(self, grad_norm_sum: Optional[torch.Tensor],
                          view_count: Optional[torch.Tensor]):
        """Make every later backward add, per Gaussian, the sum over views of
        |dL_v/dmu| to grad_norm_sum (float32, n) and the number of views that
        saw it to view_count (int32, n); None, None turns this off.  The
        tensors must stay alive while set."""
        ts = [t for t in (grad_norm_sum, view_count) if t is not None]
        if grad_norm_sum is not None and grad_norm_sum.dtype != torch.float32:
            raise ValueError("grad_norm_sum must be float32")
        if view_count is not None and view_count.dtype != torch.int32:
            raise ValueError("view_count must be int32")
        cap = min(int(t.numel()) for t in ts) if ts else 0
        self._densify_keep = ts
        L.check(self._lib.vgr_set_densify_stats(self._h, _dev_ptr(grad_norm_sum),
                                                 _dev_ptr(view_count), cap), self._h)

    def set_timing(self, on: bool):
        L.check(self._lib.vgr_set_timing(self._h, int(bool(on))), self._h)

    def timing(self) -> dict:
        cap = 16
        names = (C.c_char_p * cap)()
        ms = (C.c_float * cap)()
        cnt = C.c_int32()
        L.check(self._lib.vgr_get_timing(self._h, cap, names, ms, C.byref(cnt)), self._h)
        return {names[i].decode(): float(ms[i]) for i in range(cnt.value)}

    def _step_args(self, params, cams, settings, outs, dL, grads):
        means, quats, scales, dens, sh = params
        ncam = len(cams)
        cam_arr = (L.vgr_camera * ncam)(*[camera_struct(c) for c in cams])
        out_ptrs = (C.c_void_p * ncam)(*[o.data_ptr() for o in outs])
        dl_ptrs = None
        if dL is not None:
            dl_ptrs = (C.c_void_p * ncam)(*[g.data_ptr() for g in dL])
        st = settings.to_c()
        xray = settings.mode == "xray"
        gsh = None if (xray or grads is None) else grads[4]
        gp = [None] * 5 if grads is None else [_dev_ptr(grads[k]) for k in range(4)] + [_dev_ptr(gsh)]
        keep = (cam_arr, out_ptrs, dl_ptrs, st)
        args = (C.byref(st), int(means.shape[0]), _dev_ptr(means), _dev_ptr(quats),
                _dev_ptr(scales), _dev_ptr(dens), None if xray else _dev_ptr(sh), ncam, cam_arr,
                out_ptrs, dl_ptrs, *gp)
        return keep, args

    def graph_capture(self, params, cams, settings, outs, dL, grads, capacity_factor=1.25,
                      zero_grads=True):
        """Capture forward + backward of these exact tensors into a HIP graph
        (see vgr_graph_capture; zero_grads: the backward overwrites the
        gradients instead of adding to them).  The tensors must stay alive and
        in place."""
        self._sync_stream()
        keep, args = self._step_args(params, cams, settings, outs, dL, grads)
        self._graph_keep = (keep, params, outs, dL, grads)
        L.check(self._lib.vgr_graph_capture(self._h, *args, float(capacity_factor),
                                            int(bool(zero_grads))), self._h)

    def graph_capture_calls(self, params, cams, views_per_call, settings, outs, dL, grads,
                            capacity_factor=1.25, zero_grads=True):
        """Capture several forward + backward calls (views_per_call[k] of the
        cameras each, in order) into one HIP graph (vgr_graph_capture_calls);
        the backwards add to the same gradients."""
        self._sync_stream()
        keep, args = self._step_args(params, cams, settings, outs, dL, grads)
        vpc = (C.c_int32 * len(views_per_call))(*[int(v) for v in views_per_call])
        self._graph_keep = (keep, params, outs, dL, grads, vpc)
        # args: settings, n, 5 params, n_views, cams, outs, dL, 5 grads
        L.check(self._lib.vgr_graph_capture_calls(
            self._h, args[0], args[1], *args[2:7], len(views_per_call), vpc, *args[8:],
            float(capacity_factor), int(bool(zero_grads))), self._h)

    def graph_launch(self):
        L.check(self._lib.vgr_graph_launch(self._h), self._h)

    def graph_check(self):
        """Wait for the replays; raise VgrError(VGR_ERR_CAPACITY) on overflow."""
        k = C.c_int64()
        L.check(self._lib.vgr_graph_check(self._h, C.byref(k)), self._h)
        return int(k.value)

    def autotune(self, params, cams, settings, outs, dL=None, grads=None, iters=3):
        """Pick the fastest launch shape (tile and records per batch) for this
        workload; returns ((w, h), batch, ms per candidate)."""
        self._sync_stream()
        keep, args = self._step_args(params, cams, settings, outs, dL, grads)
        bw, bh, bb = C.c_int32(), C.c_int32(), C.c_int32()
        ms = (C.c_float * L.VGR_TUNE_CANDIDATES)()
        L.check(self._lib.vgr_autotune(self._h, *args, int(iters), C.byref(bw), C.byref(bh),
                                       C.byref(bb), ms), self._h)
        return (bw.value, bh.value), bb.value, [float(x) for x in ms]

    def tuning_text(self) -> str:
        """The tuned shapes per workload class (vgr_tune_export)."""
        n = C.c_int64()
        L.check(self._lib.vgr_tune_export(self._h, None, 0, C.byref(n)), self._h)
        buf = C.create_string_buffer(int(n.value))
        L.check(self._lib.vgr_tune_export(self._h, buf, int(n.value), C.byref(n)), self._h)
        return buf.value.decode()

    def load_tuning(self, text: str):
        """Merge shapes written by tuning_text (vgr_tune_import)."""
        L.check(self._lib.vgr_tune_import(self._h, text.encode()), self._h)

    def sort_pairs(self, keys: torch.Tensor, vals: torch.Tensor, bits: int):
        """In-place stable radix sort of (u32 key, u32 value) device pairs."""
        self._sync_stream()
        assert keys.dtype in (torch.int32, torch.uint32) and vals.dtype in (torch.int32, torch.uint32)
        rc = self._lib.vgr_sort_pairs(self._h, _dev_ptr(keys), _dev_ptr(vals), int(keys.numel()),
                                      int(bits))
        L.check(rc, self._h)

    def sort_pairs_static(self, keys: torch.Tensor, vals: torch.Tensor, bits: int):
        """The same sort without any device allocation (library-static scratch,
        at most VGR_STATIC_SORT_MAX pairs; calls overlapping on one GPU race)."""
        self._sync_stream()
        assert keys.dtype in (torch.int32, torch.uint32) and vals.dtype in (torch.int32, torch.uint32)
        rc = self._lib.vgr_sort_pairs_static(self._h, _dev_ptr(keys), _dev_ptr(vals),
                                             int(keys.numel()), int(bits))
        L.check(rc, self._h)


class _NodeToken:
    """Held by one autograd node; the context it uses stays reserved while
    the token is alive (until the backward ran or the graph was freed)."""


class _VolRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, settings, cams, means, quats, scales, dens, sh):
        outs = renderer.forward(means, quats, scales, dens, sh, cams, settings)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.token = _NodeToken()
        renderer._owner = weakref.ref(ctx.token)
        ctx.settings = settings
        ctx.save_for_backward(means, quats, scales, dens, sh if sh is not None else torch.empty(0))
        ctx.has_sh = sh is not None and settings.mode != "xray"
        return tuple(outs)

    @staticmethod
    def backward(ctx, *gouts):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError(
                "this render's context has run another forward since (the library keeps the "
                "state of the last forward only); give each render that is differentiated "
                "later its own Renderer, or let render() pick one")
        means, quats, scales, dens, sh = ctx.saved_tensors
        gm = torch.empty_like(means)
        gq = torch.empty_like(quats)
        gs = torch.empty_like(scales)
        gd = torch.empty_like(dens)
        gsh = torch.empty_like(sh) if ctx.has_sh else None
        gl = [g if g is not None else torch.zeros(s, device=means.device)
              for g, s in zip(gouts, r.shapes)]
        r.backward(gl, gm, gq, gs, gd, gsh, accumulate=False)
        r._owner = None
        return None, None, None, gm, gq, gs, gd, gsh


_POOL = {}
_POOL_LOCK = threading.Lock()


def _pooled_renderer(device: int) -> Renderer:
    """A context of this device that no live autograd node holds: contexts
    (and their workspaces) are reused from call to call instead of being
    created per render."""
    with _POOL_LOCK:
        pool = _POOL.setdefault(device, [])
        for r in pool:
            if r._owner is None or r._owner() is None:
                r._owner = None
                return r
        r = Renderer(device)
        pool.append(r)
        return r


def render(means, quats, scales, dens, sh, cams, settings: Settings = None,
           renderer: Renderer = None):
    """Differentiable render of ``cams``; returns a tuple of per-view images.

    A context keeps the state of one forward for its backward.  Without a
    ``renderer``, one is taken from a per-device pool of contexts that no
    pending autograd node holds (a node releases its context when its
    backward has run or its graph is freed), so repeated training steps reuse
    the same workspace.  A given ``renderer`` is used as is; a backward whose
    context has run another forward since raises instead of returning the
    other forward's gradients."""
    settings = settings or Settings()
    renderer = renderer or _pooled_renderer(means.device.index or 0)
    return _VolRender.apply(renderer, settings, list(cams), means.contiguous(),
                            quats.contiguous(), scales.contiguous(), dens.contiguous(),
                            None if sh is None else sh.contiguous())
