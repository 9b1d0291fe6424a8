"""MI355X (gfx950) hash-based multi-phase SpGEMM, C = A * B on CSR.

Submodules:
  spgemm   -- ctypes binding of libspgemm.so (the C ABI in include/spgemm.h)
  gen      -- seeded synthetic inputs
Importing the package loads nothing; the HIP library is loaded on first use.
"""
__all__ = ["spgemm", "gen"]
