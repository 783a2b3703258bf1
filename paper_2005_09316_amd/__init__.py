"""MI355X-native direct-Fourier visibility prediction (points, Gaussians,
shapelets) behind the C ABI of include/vp.h.

``paper_2005_09316_amd.vp`` is the ctypes binding of libvp.so; it loads the
library on first use and raises if it has not been built.
"""
from . import vp  # noqa: F401

__all__ = ["vp"]
