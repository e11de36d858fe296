"""MI355X (gfx950) implementation of FlashSplat's splat-and-accumulate path.

The compute lives in libflashsplat.so (HIP kernels behind a C ABI, declared in
include/flashsplat.h); `_lib` is its ctypes binding and `solve` drives the
calls over views. Importing this package needs torch; calling into it needs
the built library and a GPU.
"""
from . import _lib  # noqa: F401
from ._lib import (Bins, Context, DeviceScene, FlashSplatError, Proj, cameras, load, params,  # noqa: F401
                   params_exact)

__all__ = ["Bins", "Context", "DeviceScene", "FlashSplatError", "Proj", "cameras", "load", "params",
           "params_exact"]
