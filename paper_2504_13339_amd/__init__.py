"""VEG splatting rasterizer for AMD Instinct MI355X (gfx950).

The rasterizer of Volume Encoding Gaussians (arXiv 2504.13339): Gaussians carrying a scalar
value, a 1D transfer function applied per Gaussian, EWA projection, 16x16 tile binning,
front-to-back compositing, and the hand-written adjoint.  The kernels live in
``libveg.so`` (HIP, built in-tree by ``csrc/build.py``); this package is a thin ctypes
binding plus the torch-facing render / autograd / training-step helpers.  There is no CPU
fallback: importing the submodules works without a GPU, calling them needs the library
and a gfx950 device.
"""
from ._lib import LIB_PATH, VegError, load  # noqa: F401

__all__ = ["LIB_PATH", "VegError", "load", "veg", "render"]


def __getattr__(name):
    if name in ("veg", "render", "serve"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
