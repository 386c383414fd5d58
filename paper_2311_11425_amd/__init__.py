"""MI355X-native batched LHEVI vertical column solver (arXiv 2311.11425).

The product is the C-ABI library ``libhevi.so`` (HIP kernels for gfx950, see
``include/hevi.h``); ``hevi`` is its thin ctypes binding and ``inputs`` the
seeded synthetic workload generator.  Importing the package loads nothing; the
binding loads the library on first use and fails loudly if it is missing.
"""
__all__ = ["hevi", "inputs", "build"]
