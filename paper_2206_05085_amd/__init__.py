"""MI355X (gfx950) kernels of the per-ray training step of direct voxel-grid radiance
fields (Sun, Sun & Chen, arXiv 2206.05085): trilinear gathers from dense grids, the
density-to-alpha activation, front-to-back compositing, the O(N) distortion loss, the
hand-written backward with scatter-add into the grids, the fused Adam step and the colour
MLP on FP16 matrix cores with split (hi + lo) operands, which gives FP32-grade products.

The kernels live in ``libdvgo.so`` (C-ABI declared in ``include/dvgo.h``); ``ops`` is its
thin binding, ``autograd`` wraps it as torch.autograd.Function, ``step`` drives a whole
training step.  Importing this package does not load the library; the first call does,
and raises if it has not been built.
"""
from ._lib import DvgoError, lib  # noqa: F401

__all__ = ["DvgoError", "lib", "ops", "autograd", "step"]


def __getattr__(name):
    if name in ("ops", "autograd", "step"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
