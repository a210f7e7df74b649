"""Closed-form spectra of the textbook pencils built by ``pencilgen``.

These are pins that do not go through any eigen-solver: the eigenvalues are
written from their formulas.
"""
import math

import numpy as np


def fem_eigs(N=(6, 7, 8), w=(1.0, 1.3, 1.7)) -> np.ndarray:
    """Tensor linear-FEM pencil: lambda = mu^x_p + mu^y_q + mu^z_r with
    mu_p = w (6/h^2) (1 - cos p pi h) / (2 + cos p pi h), h = 1/(N+1)."""
    mus = []
    for Nd, wd in zip(N, w):
        h = 1.0 / (Nd + 1)
        p = np.arange(1, Nd + 1)
        th = p * math.pi * h
        mus.append(wd * (6.0 / h ** 2) * (1 - np.cos(th)) / (2 + np.cos(th)))
    tot = mus[0][:, None, None] + mus[1][None, :, None] + mus[2][None, None, :]
    return np.sort(tot.ravel())


def chain_eigs(n, a, b) -> np.ndarray:
    """tridiag(b, a, b): a + 2 b cos(j pi / (n + 1)), j = 1..n."""
    j = np.arange(1, n + 1)
    return np.sort(a + 2 * b * np.cos(j * math.pi / (n + 1)))


def sturm_count(n, a, b, sigma) -> int:
    """Number of eigenvalues below sigma of tridiag(b, a, b) by the Sturm
    sequence of leading principal minors (Givens)."""
    cnt = 0
    q = a - sigma
    if q < 0:
        cnt += 1
    for _ in range(1, n):
        q = (a - sigma) - b * b / q
        if q < 0:
            cnt += 1
    return cnt
