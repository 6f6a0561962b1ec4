"""RaftGP hot path on MI355X (gfx950): HIP kernels behind a C ABI
(include/raftgp.h, libraftgp.so) with a thin torch/ctypes binding.

Importing the package does not load the library; the first Context() does,
and fails loudly if libraftgp.so is missing.  There is no CPU fallback.
"""
__all__ = ["api", "build"]
