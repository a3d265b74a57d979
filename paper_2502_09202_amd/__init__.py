"""MI355X-native per-frame video measure engine (libvsa) and its Python binding.

The product is ``libvsa.so`` (HIP kernels for gfx950 + host runtime) behind the
C ABI in ``include/vsa.h``; :mod:`paper_2502_09202_amd.vsa` is the ctypes
binding with the same names.
"""
from . import vsa  # noqa: F401
