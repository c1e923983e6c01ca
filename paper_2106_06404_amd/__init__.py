"""MI355X (gfx950) multilevel spectral domain decomposition.

The compute path is libmsdd.so (HIP kernels behind the C ABI of
include/msdd.h); `binding` is a thin ctypes layer over it.
"""
