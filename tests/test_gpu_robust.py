"""Edge cases of the inertia count and of the three-stage driver on the GPU.

* pivoting restricted to a 64-column tile: a dense pencil whose pivot columns
  have their largest entries far below their tile (and tiny diagonals) still
  gives the dense count at every shift, with 2x2 pivots and the element growth
  reported by kth_factor_stats;
* 2x2 pivots occur on the tight-binding pencils (small-front and tile paths);
* a stage-1 start vector that is an exact eigenvector: the Rayleigh quotient is
  that eigenvalue (a zero pivot, so the shift moves) and the Lanczos process
  breaks down at once (beta = 0), so stage 1 restarts from the next seeded
  vector; the result still matches the dense oracle;
* a batch that names one pencil twice is rejected before any work starts.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import pencilgen as pg
from oracle import dense as od
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


def dense_pencil(n=320, nweak=96, seed=0):
    """One dense front (nf = n > 128: factored in 64-column tiles).  The first
    nweak columns have diagonals of size 1e-6 and their largest entry (about 1)
    in row i + 200, far below their pivot tile; the rest is noise of size 1e-3."""
    rng = np.random.default_rng(seed)
    X = rng.normal(scale=1e-3, size=(n, n))
    A = (X + X.T) / 2
    d = rng.uniform(-1, 1, n)
    d[:nweak] = rng.uniform(-1e-6, 1e-6, nweak)
    A[np.arange(n), np.arange(n)] = d
    for i in range(nweak):
        A[i, i + 200] = A[i + 200, i] = 1.0 + 0.1 * i / nweak
    Y = rng.normal(scale=0.02, size=(n, n))
    B = np.eye(n) + (Y @ Y.T) / n
    P = sp.csr_matrix(np.ones((n, n)))
    P.sort_indices()
    return pg.Pencil(n=n, rowptr=P.indptr.astype(np.int64), col=P.indices.astype(np.int32),
                     a_val=A.ravel().copy(), b_val=B.ravel().copy(), k=n // 2, name="tilebelow")


def test_tile_restricted_pivoting_dense_count(K, ctx):
    p = dense_pencil()
    lam = od.eigvals(p)
    note(f"tile-restricted pivoting n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    rng = np.random.default_rng(1)
    sig = np.concatenate([rng.uniform(lam[0] - 0.2, lam[-1] + 0.2, 40),
                          0.5 * (lam[1:] + lam[:-1])[::16]])
    for s in sig:
        if np.min(np.abs(lam - s)) < 1e-9:
            continue
        assert P.nu(s) == od.nu(lam, s), s
    F = P.factor(0.0)
    st = F.stats()
    assert F.inertia()[0] == od.nu(lam, 0.0)
    assert st["n2x2"] > 0
    assert 1.0 <= st["max_abs_l"] < 1e8 and st["min_pivot_rel"] > 0
    # the driver reports the growth it saw, and validates the eigenpair
    lam_k, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n))
    assert info["k_validated"] == p.k
    assert abs(lam_k - lam[p.k - 1]) <= 1e-10 * od.norm_inf(p)
    assert info["max_abs_l"] >= 1.0 and info["weak_pivot_kept"] == 0


def test_two_by_two_pivots_tight_binding(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    lam = od.eigvals(p)
    note("2x2 pivots n=2048")
    P = K.Pencil.from_pencilgen(ctx, p)
    n2 = 0
    for s in (-6.0, -3.15, -1.0, 0.5):
        F = P.factor(s)
        assert F.inertia()[0] == od.nu(lam, s)
        n2 += F.stats()["n2x2"]
    assert n2 > 0


def test_stage1_restart_from_eigenvector(K, ctx):
    base = pg.tb_supercell((3, 3, 3), seed=5)
    i0 = 17
    rows = np.repeat(np.arange(base.n), np.diff(base.rowptr))
    off = ((rows == i0) | (base.col == i0)) & (rows != base.col)
    a = base.a_val.copy()
    b = base.b_val.copy()
    a[off] = 0.0                      # row and column i0 decoupled (explicit zeros)
    b[off] = 0.0
    a[(rows == i0) & (base.col == i0)] = 1.5
    b[(rows == i0) & (base.col == i0)] = 1.0
    p = pg.Pencil(n=base.n, rowptr=base.rowptr, col=base.col, a_val=a, b_val=b, k=base.n // 2)
    lam_ref, x_ref = od.kth(p, p.k)
    assert abs(lam_ref - 1.5) > 0.1
    sv = pg.start_vectors(p.n)
    sv[0] = 0.0
    sv[0, i0] = 1.0                   # e_i0: an exact eigenvector (lambda = 1.5)
    note("stage-1 restart from an eigenvector")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=sv)
    assert info["stage1_restarts"] == 1
    assert info["weak_pivot_nudges"] >= 1      # sigma = theta_1 = 1.5 hit the zero pivot
    assert info["k_validated"] == p.k
    assert abs(lam - lam_ref) <= 1e-10 * od.norm_inf(p)
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_batch_rejects_repeated_pencil(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=3)
    note("repeated pencil in a batch")
    P = K.Pencil.from_pencilgen(ctx, p)
    Q = K.Pencil.from_pencilgen(ctx, p)
    with pytest.raises(K.KthError) as e:
        K.eig_batch(ctx, [P, Q, P], [p.k, p.k, p.k])
    assert e.value.status == K.KTH_EINVAL
    res = K.eig_batch(ctx, [P, Q], [p.k, p.k])
    assert res[0][0] == res[1][0] == K.KTH_OK
    assert res[0][1] == res[1][1]
