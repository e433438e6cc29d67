"""MI355X-native grouped Barnes-Hut oct-tree gravity (N. Nakasato, "Oct-tree
Method on GPU"): HIP kernels for gfx950 behind the C ABI in include/bh.h.

Submodules:
  bh      -- ctypes binding of libbh.so (the product path; needs the GPU)
  inputs  -- seeded synthetic particle sets
  build   -- hipcc build of libbh.so
"""
__all__ = ["bh", "inputs", "build"]
