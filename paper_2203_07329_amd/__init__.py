"""Sketch-preconditioned Tikhonov least squares on AMD MI355X (gfx950).

The method of Meier & Nakatsukasa (randomized algorithms for Tikhonov
regularization in linear least squares) as a HIP library, libtik.so, with the
C ABI declared in include/tik.h.  ``paper_2203_07329_amd.tik`` is the thin
ctypes binding; importing this package does not load the library, so the
pure-host tooling works without a GPU.
"""

__all__ = ["tik", "build"]
