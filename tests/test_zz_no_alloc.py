"""kth_solve_noalloc (the allocation-free solve) against kth_solve.

Two calls in a row on one GPU, the second with a smaller pencil than the first
(the shared work array then still holds the first call's values), each with two
right-hand sides: the allocation-free result equals the allocating solve's bit
for bit, for an FP64 factor and for one unrefined pass of an FP32 factor.
"""
import ctypes as C

import numpy as np
import pytest

import pencilgen as pg
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


def _hip():
    """The HIP runtime that libkth.so itself links (one instance per process)."""
    import glob
    h = C.CDLL(sorted(glob.glob("/opt/rocm/lib/libamdhip64.so*"))[0])
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    h.hipFree.argtypes = [C.c_void_p]
    return h


class _Dev:
    """A device copy of a host array (hipMalloc'd by the test, not the library)."""

    def __init__(self, hip, host):
        self.hip, self.nbytes = hip, host.nbytes
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), self.nbytes) == 0
        assert hip.hipMemcpy(self.p, host.ctypes.data, self.nbytes, 1) == 0

    def get(self, like):
        out = np.empty_like(like)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(out.ctypes.data, self.p, self.nbytes, 2) == 0
        return out

    def free(self):
        self.hip.hipFree(self.p)


def _solve_both(K, ctx, F, n, flags, seed):
    hip = _hip()
    b = np.asfortranarray(np.random.default_rng(seed).normal(size=(n, 2)))
    bd = _Dev(hip, b)
    xa = _Dev(hip, np.zeros_like(b))
    xb = _Dev(hip, np.full_like(b, np.nan))
    try:
        K._check(K.lib().kth_solve(F.h, 2, bd.p.value, n, xa.p.value, n,
                                   K.KTH_DEVICE_PTRS | flags), ctx.h)
        K._check(K.lib().kth_solve_noalloc(F.h, 2, bd.p.value, n, xb.p.value, n, flags), ctx.h)
        return xa.get(b), xb.get(b)
    finally:
        for d in (bd, xa, xb):
            d.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_noalloc_matches_solve(prec):
    K = kth()
    ctx = K.Context(0)
    precision = K.KTH_FP64 if prec == "fp64" else K.KTH_FP32_IR
    flags = 0 if prec == "fp64" else K.KTH_SOLVE_UNREFINED
    for cells, sigma, seed in (((4, 4, 4), -3.1, 0), ((2, 2, 3), -2.0, 1)):
        p = pg.tb_supercell(cells, seed=seed)
        note(f"kth_solve_noalloc {prec} n={p.n}")
        P = K.Pencil.from_pencilgen(ctx, p)
        F = P.factor(sigma, precision)
        xa, xb = _solve_both(K, ctx, F, p.n, flags, seed)
        assert np.isfinite(xa).all()
        assert np.array_equal(xa, xb)
        if prec == "fp64":
            C_ = p.A() - sigma * p.B()
            b = np.random.default_rng(seed).normal(size=(p.n, 2))
            assert np.linalg.norm(C_ @ xb - b) <= 1e-10 * np.linalg.norm(b)
        F.close()
        P.close()


def test_solve_noalloc_rejects_refined_fp32():
    K = kth()
    ctx = K.Context(0)
    p = pg.tb_supercell((2, 2, 2), seed=2)
    note("kth_solve_noalloc refused for a refined FP32 solve")
    P = K.Pencil.from_pencilgen(ctx, p)
    F = P.factor(-2.0, K.KTH_FP32_IR)
    hip = _hip()
    b = _Dev(hip, np.ones(p.n))
    x = _Dev(hip, np.zeros(p.n))
    try:
        st = K.lib().kth_solve_noalloc(F.h, 1, b.p.value, p.n, x.p.value, p.n, 0)
        assert st == K.KTH_EINVAL
    finally:
        b.free()
        x.free()


def test_solve_noalloc_headline_size():
    # the n = 524288 workload's factor fits the fixed work array
    K = kth()
    ctx = K.Context(0)
    p = pg.workload("n524k")
    note("kth_solve_noalloc n=524288")
    P = K.Pencil.from_pencilgen(ctx, p)
    F = P.factor(-3.0)
    xa, xb = _solve_both(K, ctx, F, p.n, 0, 3)
    assert np.array_equal(xa, xb)
