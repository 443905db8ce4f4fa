"""MI355X-native 25-point star stencil / acoustic leapfrog library.

The compute path is libstencil.so (hand-written HIP for gfx950) behind the
C ABI in include/stencil.h; ``lib`` is its ctypes binding.  Submodules are
imported on demand so that the CPU-only parts (layout, ABI checks) work
without a GPU.
"""

__all__ = ["lib", "fields", "build"]
