"""MI355X-native semismooth Newton solver for the kernel-based OT estimator (arXiv 2310.14087).

* ``kotssn``  — ctypes binding of the C-ABI library ``libkotssn.so`` (HIP kernels for gfx950).
* ``inputs``  — seeded synthetic problem generator.
* ``build``   — in-tree hipcc build of the library.
"""
__all__ = ["kotssn", "inputs", "build"]
