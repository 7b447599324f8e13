"""MI355X-native FFT-preconditioned FE homogenization solver.

The solver lives in libfh.so (HIP kernels for gfx950 + a C-ABI, see
include/fh.h); this package holds its sources (csrc/), the build script and
a thin ctypes binding (fh.py).
"""
from .fh import Context, load_library, FHError  # noqa: F401
