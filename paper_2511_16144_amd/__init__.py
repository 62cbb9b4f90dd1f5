"""MI355X (gfx950) differentiable Gaussian rasterizer: RGB + depth + 16-d
language feature, forward and backward, behind the C ABI of
``include/lego_raster.h`` (``liblego_raster.so``, built by ``build_lib.py``).

The package holds the HIP sources (``csrc/``), the build script and the ctypes
binding; it has no CPU fallback.
"""
from .binding import (Context, State, Settings, RasterFn, render, LgsError, load_library, lib,
                      EXPORTS, LIB_PATH)
from .params import params_from_arrays

__all__ = ["Context", "State", "Settings", "RasterFn", "render", "LgsError", "load_library", "lib",
           "EXPORTS", "LIB_PATH", "params_from_arrays"]
