"""MI355X-native soft demapping and Monte-Carlo MI/GMI estimation (libair).

Submodules:
  inputs  seeded synthetic workloads (no method arithmetic)
  air     thin ctypes binding to the HIP library libair.so (C ABI in include/air.h)
  build   compiles libair.so for gfx950 with hipcc
"""
__all__ = ["inputs", "air", "build"]
