"""Operand layout of v_mfma_f64_16x16x4 on gfx950, pinned by a raw probe.

The Schur-update kernel feeds lane l with A(m = l % 16, k = l / 16) and
B(k = l / 16, n = l % 16) and reads result register r of lane l as
D(m = 4 r + l / 16, n = l % 16); this test pins that layout.
"""
import itertools

import numpy as np
import pytest

from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu

A_MAPS = {"m=l%16,k=l/16": lambda l: (l % 16, l // 16), "m=l/4,k=l%4": lambda l: (l // 4, l % 4)}
B_MAPS = {"n=l%16,k=l/16": lambda l: (l // 16, l % 16), "n=l/4,k=l%4": lambda l: (l % 4, l // 4)}
D_MAPS = {
    "m=4(l/16)+r,n=l%16": lambda l, r: (4 * (l // 16) + r, l % 16),
    "m=l%16,n=4(l/16)+r": lambda l, r: (l % 16, 4 * (l // 16) + r),
    "m=4r+l/16,n=l%16": lambda l, r: (4 * r + l // 16, l % 16),
    "m=l%16,n=4r+l/16": lambda l, r: (l % 16, 4 * r + l // 16),
}


def identify(a, b, d, tol=1e-13):
    found = []
    for (an, am), (bn, bm), (dn, dm) in itertools.product(A_MAPS.items(), B_MAPS.items(), D_MAPS.items()):
        A = np.zeros((16, 4)); B = np.zeros((4, 16))
        for l in range(64):
            A[am(l)] = a[l]
            B[bm(l)] = b[l]
        C = A @ B
        pred = np.array([C[dm(l, r)] for l in range(64) for r in range(4)])
        if np.allclose(pred, d, rtol=tol, atol=tol):
            found.append((an, bn, dn))
    return found


def test_mfma_f64_16x16x4_layout():
    K = kth()
    rng = np.random.default_rng(0)
    a = rng.normal(size=64)
    b = rng.normal(size=64)
    note("mfma raw probe")
    d = K.kth_debug_mfma_probe(a, b)
    found = identify(a, b, d)
    print("layouts matching:", found)
    assert found == [("m=l%16,k=l/16", "n=l%16,k=l/16", "m=4r+l/16,n=l%16")], found


def test_mfma_f32_16x16x4_layout():
    """The FP32 instruction used by the FP32 shift-and-invert factor."""
    K = kth()
    rng = np.random.default_rng(1)
    a = rng.normal(size=64).astype(np.float32)
    b = rng.normal(size=64).astype(np.float32)
    note("mfma f32 raw probe")
    d = K.kth_debug_mfma_probe_f32(a, b).astype(np.float64)
    found = identify(a.astype(np.float64), b.astype(np.float64), d, tol=1e-5)
    print("f32 layouts matching:", found)
    # FP32 differs from FP64: register r of lane l holds row 4 (l / 16) + r
    assert found == [("m=l%16,k=l/16", "n=l%16,k=l/16", "m=4(l/16)+r,n=l%16")], found
