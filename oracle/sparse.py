"""Oracle (test infrastructure only): ctypes wrapper of the plain-C sparse LDL^T.

``inertia(pencil, sigma)`` returns (neg, zero, pos) of A - sigma B, i.e. by
Sylvester's law (Section 2.1) nu_sigma(A, B) = neg when zero == 0.
``Factor`` keeps L, D for solves (the linear systems of Alg. 2 and Alg. 3).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build
from .ordering import coordinate_nd


class Stats(C.Structure):
    _fields_ = [("neg", C.c_int64), ("zero", C.c_int64), ("pos", C.c_int64),
                ("min_abs_d", C.c_double), ("max_abs_l", C.c_double),
                ("flops", C.c_double), ("flops_done", C.c_double),
                ("nnz_l", C.c_int64), ("nsuper", C.c_int64), ("max_front", C.c_int64),
                ("n2x2", C.c_int64), ("completed", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(os.path.dirname(_build.LIB), "ldlt.c")
        if (not os.path.exists(_build.LIB)
                or os.path.getmtime(_build.LIB) < os.path.getmtime(src)):
            _build.build()
        L = C.CDLL(_build.LIB)
        p64, pi32, pd = C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
        L.orc_ldlt.argtypes = [C.c_int64, p64, pi32, pd, pd, C.c_double, p64, C.c_int,
                               C.c_double, C.POINTER(Stats), C.POINTER(C.c_void_p), p64]
        L.orc_front_sample.argtypes = [C.c_int64, C.c_int64, C.c_int64, pd, pd]
        L.orc_front_sample.restype = C.c_int
        L.orc_ldlt.restype = C.c_int
        L.orc_solve.argtypes = [C.c_void_p, pd, pd]
        L.orc_solve.restype = C.c_int
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_free.restype = None
        L.orc_shifted_matvec.argtypes = [C.c_int64, p64, pi32, pd, pd, C.c_double, pd, pd]
        L.orc_shifted_matvec.restype = None
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class _Arrays:
    """Keeps contiguous copies of a pencil's arrays alive across calls."""

    def __init__(self, pencil, perm=None):
        self.n = int(pencil.n)
        self.rowptr = np.ascontiguousarray(pencil.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(pencil.col, dtype=np.int32)
        self.a = np.ascontiguousarray(pencil.a_val, dtype=np.float64)
        self.b = np.ascontiguousarray(pencil.b_val, dtype=np.float64)
        if perm is None:
            perm = coordinate_nd(self.rowptr, self.col, getattr(pencil, "coords", None))
        self.perm = np.ascontiguousarray(perm, dtype=np.int64)


def prepare(pencil, perm=None) -> _Arrays:
    return pencil if isinstance(pencil, _Arrays) else _Arrays(pencil, perm)


def ldlt_stats(pencil, sigma: float, flop_cap: float = 0.0) -> Stats:
    """Factor A - sigma B (without keeping L) and return the statistics."""
    P = prepare(pencil)
    st = Stats()
    rc = lib().orc_ldlt(P.n, _ptr(P.rowptr, C.c_int64), _ptr(P.col, C.c_int32),
                        _ptr(P.a, C.c_double), _ptr(P.b, C.c_double), float(sigma),
                        _ptr(P.perm, C.c_int64), 0, float(flop_cap), C.byref(st), None, None)
    if rc != 0:
        raise ValueError("oracle LDL^T rejected its input")
    return st


def front_shapes(pencil):
    """(nf, ns) of every supernode of the oracle's own symbolic analysis, in
    elimination order (int64 array of shape (nsuper, 2)), and the flop total."""
    P = prepare(pencil)
    st = Stats()
    shapes = np.zeros(2 * P.n, dtype=np.int64)
    rc = lib().orc_ldlt(P.n, _ptr(P.rowptr, C.c_int64), _ptr(P.col, C.c_int32),
                        _ptr(P.a, C.c_double), _ptr(P.b, C.c_double), 0.0,
                        _ptr(P.perm, C.c_int64), 0, 1.0, C.byref(st), None,
                        _ptr(shapes, C.c_int64))
    if rc != 0:
        raise ValueError("oracle LDL^T rejected its input")
    return shapes[: 2 * st.nsuper].reshape(-1, 2), float(st.flops)


def front_sample(nf: int, ns: int, cap: int = 0) -> tuple[float, float]:
    """(seconds, flops) of the oracle's partial factorization of one synthetic
    dense front (timing sample for the CPU baseline; see orc_front_sample)."""
    secs, fl = C.c_double(), C.c_double()
    if lib().orc_front_sample(int(nf), int(ns), int(cap), C.byref(secs), C.byref(fl)) != 0:
        raise ValueError("bad front shape")
    return secs.value, fl.value


def inertia(pencil, sigma: float) -> tuple[int, int, int]:
    st = ldlt_stats(pencil, sigma)
    return int(st.neg), int(st.zero), int(st.pos)


def nu(pencil, sigma: float) -> int:
    """nu_sigma(A, B): number of eigenvalues below sigma (Section 2.1)."""
    neg, zero, _ = inertia(pencil, sigma)
    if zero:
        raise ZeroDivisionError(f"sigma={sigma!r} gives a zero pivot (singular A - sigma B)")
    return neg


class Factor:
    """Kept LDL^T factor of A - sigma B with ``solve``."""

    def __init__(self, pencil, sigma: float):
        self.P = prepare(pencil)
        self.sigma = float(sigma)
        self.stats = Stats()
        h = C.c_void_p()
        P = self.P
        rc = lib().orc_ldlt(P.n, _ptr(P.rowptr, C.c_int64), _ptr(P.col, C.c_int32),
                            _ptr(P.a, C.c_double), _ptr(P.b, C.c_double), self.sigma,
                            _ptr(P.perm, C.c_int64), 1, 0.0, C.byref(self.stats), C.byref(h), None)
        if rc != 0 or not h.value:
            raise ValueError("oracle LDL^T failed")
        self._h = h

    @property
    def inertia(self):
        s = self.stats
        return int(s.neg), int(s.zero), int(s.pos)

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        lib().orc_solve(self._h, _ptr(b, C.c_double), _ptr(x, C.c_double))
        return x

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.orc_free(h)
            self._h = None


def shifted_matvec(pencil, sigma: float, x: np.ndarray) -> np.ndarray:
    P = prepare(pencil)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().orc_shifted_matvec(P.n, _ptr(P.rowptr, C.c_int64), _ptr(P.col, C.c_int32),
                             _ptr(P.a, C.c_double), _ptr(P.b, C.c_double), float(sigma),
                             _ptr(x, C.c_double), _ptr(y, C.c_double))
    return y
