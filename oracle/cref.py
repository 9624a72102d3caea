"""ctypes wrapper of the matrix-free C oracle c/ddref.c (test infrastructure only).

The C oracle covers lattices too large for the assembled sparse matrix
(48x24^3 and up) and is timed as the CPU baseline.  It is built by ``build()``
with gcc (plain -O3 and OpenMP, no intrinsics).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "ddref.c")
LIB = os.path.join(HERE, "c", "libddref.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.ref_create.restype = P
        L.ref_create.argtypes = [P, P, I, D, P]
        L.ref_destroy.argtypes = [P]
        L.ref_clover.argtypes = [P, P]
        L.ref_dslash.argtypes = [P, D, P, P]
        L.ref_block_apply.argtypes = [P, I, D, P, P]
        L.ref_hop.argtypes = [P, I, P, P]
        L.ref_solve.argtypes = [P, D, P, P, D, I]
        L.ref_solve.restype = I
        L.ref_block_solve.argtypes = [P, I, D, P, P, D, I]
        L.ref_block_solve.restype = I
        L.ref_schur_apply.argtypes = [P, D, P, P, D]
        L.ref_schur_apply.restype = I
        L.ref_schur_inverse.argtypes = [P, D, P, P, D]
        L.ref_schur_inverse.restype = I
        L.ref_exponent.argtypes = [P, I, I, D, D, P, D, ctypes.POINTER(ctypes.c_double)]
        L.ref_exponent.restype = I
        L.ref_record.argtypes = [I, I, P, P]
        L.ref_record.restype = I
        L.ref_threads.restype = I
        L.ref_set_threads.argtypes = [I]
        L.ref_set_threads.restype = None
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class CRef:
    """Matrix-free FP64 oracle on one gauge field."""

    def __init__(self, links, lat, blk, csw: float, time_bc: int = -1):
        self.L = _load()
        self.lat = tuple(int(v) for v in lat)
        self.V = int(np.prod(self.lat))
        self._lat = np.array(self.lat, dtype=np.int32)
        self._blk = np.array(blk, dtype=np.int32)
        self._links = _c(links)
        self.h = self.L.ref_create(self._lat.ctypes.data, self._blk.ctypes.data, int(time_bc), float(csw),
                                   self._links.ctypes.data)

    def close(self):
        if self.h:
            self.L.ref_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _out(self):
        return np.zeros((self.V, 4, 3), dtype=np.complex128)

    def clover(self):
        out = np.zeros((self.V, 12, 12), dtype=np.complex128)
        self.L.ref_clover(self.h, out.ctypes.data)
        return out

    def dslash(self, m, psi):
        psi = _c(psi)
        out = self._out()
        self.L.ref_dslash(self.h, float(m), psi.ctypes.data, out.ctypes.data)
        return out

    def block_apply(self, colour, m, psi):
        psi = _c(psi)
        out = self._out()
        self.L.ref_block_apply(self.h, int(colour), float(m), psi.ctypes.data, out.ctypes.data)
        return out

    def hop(self, to_colour, psi):
        psi = _c(psi)
        out = self._out()
        self.L.ref_hop(self.h, int(to_colour), psi.ctypes.data, out.ctypes.data)
        return out

    def solve(self, m, b, tol=1e-13, maxit=100000):
        b = _c(b)
        x = self._out()
        it = self.L.ref_solve(self.h, float(m), b.ctypes.data, x.ctypes.data, float(tol), int(maxit))
        if it < 0:
            raise RuntimeError("C oracle solve did not converge")
        return x

    def block_solve(self, colour, m, b, tol=1e-13, maxit=100000):
        b = _c(b)
        x = self._out()
        it = self.L.ref_block_solve(self.h, int(colour), float(m), b.ctypes.data, x.ctypes.data, float(tol), int(maxit))
        if it < 0:
            raise RuntimeError("C oracle block solve did not converge")
        return x

    def schur_apply(self, m, phi, tol=1e-13):
        phi = _c(phi)
        out = self._out()
        if self.L.ref_schur_apply(self.h, float(m), phi.ctypes.data, out.ctypes.data, float(tol)):
            raise RuntimeError("C oracle block solve did not converge")
        return out

    def schur_inverse(self, m, phi, tol=1e-13):
        phi = _c(phi)
        out = self._out()
        if self.L.ref_schur_inverse(self.h, float(m), phi.ctypes.data, out.ctypes.data, float(tol)):
            raise RuntimeError("C oracle solve did not converge")
        return out

    def exponent_recorded(self, op, form, m1, m2, eta, tol=1e-13, cap=0):
        """exponent() with the solves' iterations and seconds recorded (each capped at `cap`
        iterations when cap > 0, which gives a timing sample, not a converged result)."""
        self.L.ref_record(1, int(cap), None, None)
        eta = _c(eta)
        x = ctypes.c_double()
        self.L.ref_exponent(self.h, 0 if op == "full" else 1, 0 if form == "plain" else 1, float(m1), float(m2),
                            eta.ctypes.data, float(tol), ctypes.byref(x))
        iters = np.zeros(16, dtype=np.int32)
        secs = np.zeros(16)
        n = self.L.ref_record(0, 0, iters.ctypes.data, secs.ctypes.data)
        return x.value, iters[:n].tolist(), secs[:n].tolist()

    @staticmethod
    def threads() -> int:
        return int(_load().ref_threads())

    @staticmethod
    def set_threads(n: int) -> None:
        """Thread count of the oracle's OpenMP regions from now on (timing only)."""
        _load().ref_set_threads(int(n))

    def exponent(self, op: str, form: str, m1, m2, eta, tol=1e-13) -> float:
        eta = _c(eta)
        x = ctypes.c_double()
        st = self.L.ref_exponent(self.h, 0 if op == "full" else 1, 0 if form == "plain" else 1, float(m1), float(m2),
                                 eta.ctypes.data, float(tol), ctypes.byref(x))
        if st:
            raise RuntimeError("C oracle solve did not converge")
        return x.value
