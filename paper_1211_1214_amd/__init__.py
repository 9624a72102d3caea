"""Schwarz-factorised stochastic determinant ratios for Wilson-clover fermions on MI355X.

The computation lives in libddwc.so (HIP kernels for gfx950 behind the C ABI of
include/ddwc.h); ``binding`` is its ctypes wrapper and ``inputs`` the seeded
synthetic input generators.  Importing the package loads nothing; the library is
loaded on first use and its absence is an error.
"""
from .binding import (BLACK, FP64, MIXED16, MIXED32, OP_FULL, OP_SCHUR, WHITE, Context, DDWCError,  # noqa: F401
                      lib, mass)

__all__ = ["Context", "DDWCError", "lib", "mass", "FP64", "MIXED32", "MIXED16", "BLACK", "WHITE", "OP_FULL", "OP_SCHUR"]
