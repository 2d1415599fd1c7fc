"""Volumetrically consistent 3D Gaussian rasterisation (arXiv 2412.03378) on
MI355X: HIP kernels behind the C ABI of include/vgr.h, with a thin PyTorch
binding.

    from paper_2412_03378_amd import Renderer, Settings, render, scenes

``scenes`` (seeded synthetic workloads) needs only numpy; the renderer
symbols load libvgr.so on first use and fail loudly if it is not built.
"""
import importlib

__all__ = ["Renderer", "Settings", "render", "camera_struct", "scenes", "build"]

_RENDERER_NAMES = ("Renderer", "Settings", "render", "camera_struct")


def __getattr__(name):
    if name in _RENDERER_NAMES:
        return getattr(importlib.import_module(".renderer", __name__), name)
    if name == "build":
        return importlib.import_module(".build", __name__).build
    if name in ("scenes", "renderer", "_lib"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
