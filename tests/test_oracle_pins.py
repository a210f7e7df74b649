"""The oracle pinned to values that do not come from itself.

* closed-form spectra (tensor FEM pencil, Toeplitz chain), Sturm counts;
* block-diagonal pencils reduce to per-block dense problems;
* Sylvester's law: nu from the sparse LDL^T equals the count of eigenvalues
  below sigma (Section 2.1), and neg + zero + pos = n; nu is non-decreasing;
* solve residuals; Hellmann-Feynman gradient vs finite differences.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import pencilgen as pg
from oracle import dense as od
from oracle import sparse as osp
from tests.closed_form import chain_eigs, fem_eigs, sturm_count


def test_dense_fem_closed_form():
    N, w = (5, 6, 7), (1.0, 1.3, 1.7)
    p = pg.fem_tensor(N, w)
    lam, X = od.eig(p)
    ref = fem_eigs(N, w)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-9 * ref.max())
    # B-orthonormal eigenvectors and residuals
    A, B = od.densify(p)
    assert np.allclose(X.T @ B @ X, np.eye(p.n), atol=1e-10)
    assert np.abs(A @ X - B @ X * lam).max() < 1e-9 * ref.max()


def test_dense_chain_closed_form():
    p = pg.chain(50, 0.3, -0.7)
    lam, _ = od.eig(p)
    assert np.allclose(lam, chain_eigs(50, 0.3, -0.7), atol=1e-13)


def test_dense_block_diag_reduces_to_blocks():
    p = pg.block_diag_perm((4, 9, 6, 3), seed=3)
    lam, _ = od.eig(p)
    ref = np.sort(np.concatenate([sla.eigh(a, b, eigvals_only=True) for a, b in p.blocks]))
    assert np.allclose(lam, ref, atol=1e-12)


def test_dense_kth_sign_and_normalisation():
    p = pg.tb_supercell((2, 2, 2), seed=4)
    lam, x = od.kth(p, 17)
    B = p.B()
    assert abs(x @ (B @ x) - 1) < 1e-12
    assert x[np.argmax(np.abs(x))] > 0


@pytest.mark.parametrize("N,w", [((6, 7, 8), (1.0, 1.3, 1.7)), ((9, 5, 4), (1.0, 0.7, 2.1))])
def test_sparse_inertia_fem_closed_form(N, w):
    p = pg.fem_tensor(N, w)
    ref = fem_eigs(N, w)
    rng = np.random.default_rng(0)
    # shifts away from eigenvalues (relative gap check) spanning the spectrum
    sig = np.concatenate([rng.uniform(ref[0] * 0.5, ref[-1] * 1.05, 40), [0.0, ref[-1] * 2]])
    P = osp.prepare(p)
    for s in sig:
        if np.min(np.abs(ref - s)) < 1e-9 * ref[-1]:
            continue
        neg, zero, pos = osp.inertia(P, s)
        assert zero == 0
        assert neg == int(np.sum(ref < s)), s
        assert neg + zero + pos == p.n


def test_sparse_inertia_chain_sturm():
    n, a, b = 200, 0.1, -1.0
    p = pg.chain(n, a, b)
    for s in np.linspace(-2.3, 2.3, 37):
        assert osp.nu(p, s) == sturm_count(n, a, b, s) == int(np.sum(chain_eigs(n, a, b) < s))


def test_sparse_inertia_block_diag():
    p = pg.block_diag_perm((7, 11, 5, 13, 2), seed=5)
    ref = np.sort(np.concatenate([sla.eigh(a, b, eigvals_only=True) for a, b in p.blocks]))
    for s in np.linspace(ref[0] - 1, ref[-1] + 1, 41):
        assert osp.nu(p, s) == int(np.sum(ref < s))


@pytest.mark.parametrize("cells,seed", [((2, 2, 2), 1), ((3, 2, 2), 2), ((4, 4, 4), 0)])
def test_sparse_inertia_tb_matches_dense_count(cells, seed):
    p = pg.tb_supercell(cells, seed=seed)
    lam, _ = od.eig(p)
    P = osp.prepare(p)
    rng = np.random.default_rng(seed)
    sig = rng.uniform(lam[0] - 0.5, lam[-1] + 0.5, 25)
    prev = -1
    n2 = 0
    for s in np.sort(sig):
        st = osp.ldlt_stats(P, s)
        assert st.zero == 0 and st.neg + st.pos == p.n
        assert st.neg == od.nu(lam, s)
        assert st.neg >= prev          # nu is non-decreasing
        prev = st.neg
        n2 += st.n2x2
    assert n2 > 0                      # the 2x2 pivot path was exercised


def test_sparse_zero_pivot_detected():
    # diagonal pencil, sigma exactly an eigenvalue: a pivot is exactly zero
    n = 10
    p = pg.Pencil(n=n, rowptr=np.arange(n + 1, dtype=np.int64), col=np.arange(n, dtype=np.int32),
                  a_val=np.arange(1.0, n + 1), b_val=np.ones(n))
    assert osp.inertia(p, 4.0) == (3, 1, 6)
    assert osp.inertia(p, 4.5) == (4, 0, 6)


def test_sparse_solve_residual():
    p = pg.tb_supercell((3, 3, 3), seed=2)
    F = osp.Factor(p, -2.5)
    b = np.random.default_rng(0).normal(size=p.n)
    x = F.solve(b)
    C = p.A() - (-2.5) * p.B()
    assert np.linalg.norm(C @ x - b) <= 1e-10 * np.linalg.norm(b)
    # FEM pencil, indefinite shift
    q = pg.fem_tensor((6, 7, 8))
    sig = 0.5 * (fem_eigs()[100] + fem_eigs()[101])
    F = osp.Factor(q, sig)
    x = F.solve(np.ones(q.n))
    C = q.A() - sig * q.B()
    assert np.linalg.norm(C @ x - 1) <= 1e-9 * math.sqrt(q.n)


def test_sparse_shifted_matvec_single_rounding():
    p = pg.tb_supercell((2, 2, 2), seed=9)
    x = np.random.default_rng(1).normal(size=p.n)
    s = -1.2345678901234
    y = osp.shifted_matvec(p, s, x)
    ref = (p.A() - s * p.B()) @ x
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_hf_gradient_matches_finite_differences():
    p = pg.tb_supercell((2, 2, 2), seed=6)
    k = p.n // 2
    lam, x = od.kth(p, k)
    gA, gB = od.hf_gradient(p, lam, x)
    # homogeneity: sum g_A a = lambda, sum g_B b = -lambda
    assert abs(np.dot(gA, p.a_val) - lam) < 1e-12 * max(1, abs(lam))
    assert abs(np.dot(gB, p.b_val) + lam) < 1e-12 * max(1, abs(lam))
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    rng = np.random.default_rng(0)
    h = 1e-6
    picks = rng.choice(np.nonzero(rows <= p.col)[0], 12, replace=False)
    for q in picks:
        i, j = rows[q], p.col[q]
        # the symmetric partner entry
        lo, hi = p.rowptr[j], p.rowptr[j + 1]
        q2 = lo + int(np.searchsorted(p.col[lo:hi], i))
        for which in ("a", "b"):
            vals = []
            for sgn in (+1, -1):
                pp = pg.Pencil(n=p.n, rowptr=p.rowptr, col=p.col, a_val=p.a_val.copy(),
                               b_val=p.b_val.copy())
                arr = pp.a_val if which == "a" else pp.b_val
                arr[q] += sgn * h
                if q2 != q:
                    arr[q2] += sgn * h
                vals.append(od.kth(pp, k)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            g = gA if which == "a" else gB
            an = g[q] + (g[q2] if q2 != q else 0.0)
            assert abs(fd - an) <= 1e-7 + 1e-5 * abs(an), (which, i, j, fd, an)


def test_norm_inf_hand_computed():
    # rows of A: |1| + |-2| + |0| = 3, |-2| + |3| + |4| = 9, |0| + |4| + |-6| = 10
    rowptr = np.array([0, 3, 6, 9], dtype=np.int64)
    col = np.array([0, 1, 2] * 3, dtype=np.int32)
    a = np.array([1.0, -2.0, 0.0, -2.0, 3.0, 4.0, 0.0, 4.0, -6.0])
    p = pg.Pencil(n=3, rowptr=rowptr, col=col, a_val=a, b_val=np.eye(3).ravel())
    assert od.norm_inf(p) == 10.0
    # a pattern with rows of different lengths (and an empty off-diagonal part)
    q = pg.chain(5, 0.5, -1.25)        # rows: 1.75, 3.0, 3.0, 3.0, 1.75
    assert od.norm_inf(q) == 3.0


def test_dense_eigvals_closed_form():
    N, w = (5, 4, 6), (1.0, 2.1, 0.6)
    ref = fem_eigs(N, w)
    lam = od.eigvals(pg.fem_tensor(N, w))
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-9 * ref.max())
    p = pg.block_diag_perm((6, 3, 8), seed=11)
    blk = np.sort(np.concatenate([sla.eigh(a, b, eigvals_only=True) for a, b in p.blocks]))
    assert np.allclose(od.eigvals(p), blk, atol=1e-12)


def test_stored_oracle_isolation_tiny():
    """The oracle-only isolation job (multisection -> shift-and-invert Lanczos ->
    inertia certificate) on the small workload, against the dense definition."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "kth_oracle_tiny.json")
    g = json.load(open(path))
    p = pg.workload("tiny")
    lam = od.eigvals(p)
    assert g["k"] == p.k and g["phase"] == "done" and g["certificate"]["holds"]
    assert abs(g["lam"] - lam[p.k - 1]) <= 1e-12 * od.norm_inf(p)
    for s, nu, zero in g["counts"]:
        assert zero == 0 and nu == od.nu(lam, s)
    c = g["certificate"]
    assert c["sigma_minus"] <= lam[p.k - 1] < c["sigma_plus"]
