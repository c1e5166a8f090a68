"""MI355X (gfx950) Winograd / Toom-Cook convolution with arbitrary points.

The method is that of arXiv:2201.10369: Winograd convolution whose transform
matrices are generated from a chosen set of interpolation points (including
the {0, inf, +-c, +-1/c} families), scored by its float32 error against a
float64 direct convolution.  All computation runs in the HIP library
libwg.so (C ABI in include/wg.h); `wg` is its Python binding.
"""
from . import wg  # noqa: F401

__all__ = ["wg"]
