"""Hemispherical ray-casting accessibility on MI355X (gfx950).

`hra` is the ctypes binding of libhra.so (HIP kernels behind a C ABI, see
include/hra.h); `build` compiles the library in-tree with hipcc.
"""
__all__ = ["hra", "build"]
