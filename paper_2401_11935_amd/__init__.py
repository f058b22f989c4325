"""MI355X-native two-determinant DCSD / CCSD amplitude residual (libdcsd).

The compute path is the HIP shared library ``libdcsd.so`` built from
``csrc/`` for gfx950; ``paper_2401_11935_amd.libdcsd`` is a thin ctypes
binding with the same names as the C ABI in ``include/libdcsd.h``.  Importing
the package does not load the library; ``libdcsd.load()`` does, and raises if
it has not been built.
"""

__all__ = ["libdcsd"]
