"""Oracle (test infrastructure only): the dense path.

The k-th eigenpair by its plain definition (eq. (1): A x = lambda B x,
eigenvalues ascending, k 1-based), computed by Cholesky reduction of the pencil
to a standard symmetric problem and a symmetric eigensolver -- the route of
the dense LAPACK generalized solver used for comparison in Section 4.2:

  B = R R^T,  C = R^{-1} A R^{-T},  C = Q Lambda Q^T,  X = R^{-T} Q  (B-orthonormal).

nu_sigma(A, B) = #{i : lambda_i < sigma} (Section 2.1).
The Hellmann-Feynman gradient of a simple lambda_k with B-normalised x_k is
d lambda / dA_ij = x_i x_j and d lambda / dB_ij = -lambda x_i x_j.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotPositiveDefinite(ValueError):
    pass


def densify(pencil):
    A = pencil.A().toarray()
    B = pencil.B().toarray()
    if not (np.array_equal(A, A.T) and np.array_equal(B, B.T)):
        raise ValueError("pencil is not symmetric")
    return A, B


def eig(pencil):
    """All eigenvalues (ascending) and B-orthonormal eigenvectors (columns)."""
    A, B = densify(pencil)
    try:
        R = np.linalg.cholesky(B)            # B = R R^T, R lower
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e))
    Y = sla.solve_triangular(R, A, lower=True)            # R^{-1} A
    Cm = sla.solve_triangular(R, Y.T, lower=True).T       # R^{-1} A R^{-T}
    Cm = 0.5 * (Cm + Cm.T)
    lam, Q = np.linalg.eigh(Cm)
    X = sla.solve_triangular(R.T, Q, lower=False)          # R^{-T} Q
    return lam, X


def eigvals(pencil):
    """All eigenvalues (ascending) by the same Cholesky reduction, without
    eigenvectors (the symmetric eigenvalue-only driver)."""
    A, B = densify(pencil)
    try:
        R = np.linalg.cholesky(B)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e))
    Y = sla.solve_triangular(R, A, lower=True)
    Cm = sla.solve_triangular(R, Y.T, lower=True).T
    return np.linalg.eigvalsh(0.5 * (Cm + Cm.T))


def sign_fix(x: np.ndarray) -> np.ndarray:
    """Largest-magnitude component made positive (first one on ties)."""
    i = int(np.argmax(np.abs(x)))
    return x if x[i] >= 0 else -x


def kth(pencil, k: int):
    """(lambda_k, x_k) with x_k^T B x_k = 1 and its largest-|.| entry positive."""
    lam, X = eig(pencil)
    return float(lam[k - 1]), sign_fix(X[:, k - 1].copy())


def nu(eigs: np.ndarray, sigma: float) -> int:
    return int(np.count_nonzero(np.asarray(eigs) < sigma))


def hf_gradient(pencil, lam: float, x: np.ndarray):
    """Gradients of a simple eigenvalue w.r.t. each stored entry value of A and B."""
    rows = np.repeat(np.arange(pencil.n), np.diff(pencil.rowptr))
    xx = x[rows] * x[pencil.col]
    return xx, -lam * xx


def norm_inf(pencil) -> float:
    """||A||_inf = max absolute row sum."""
    a = np.abs(pencil.a_val)
    return float(np.add.reduceat(a, pencil.rowptr[:-1]).max()) if pencil.nnz else 0.0
