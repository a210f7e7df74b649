"""Multiple eigenvalues on the GPU: the block shift-and-invert Lanczos.

* a pencil whose every eigenvalue is exactly double (the direct sum of a
  tight-binding cluster with itself): the single-vector Alg. 3 cannot validate
  the interval (it sees one copy of each double eigenvalue) and stops with an
  error; the automatic mode hands over to the block method, whose result
  matches the dense definition and the oracle's block run;
* the block method on a pencil with simple eigenvalues agrees with Alg. 3.
"""
import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from oracle import three_stage as o3
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


@pytest.fixture(scope="module")
def doubled():
    q = pg.doubled(pg.tb_cluster(200, seed=4), seed=None)
    return q, od.eigvals(q)


@pytest.mark.parametrize("kk", ["mid", "mid+1", "241"])
def test_double_eigenvalues_block(K, ctx, doubled, kk):
    q, lam = doubled
    k = {"mid": q.n // 2, "mid+1": q.n // 2 + 1, "241": 241}[kk]
    nA = od.norm_inf(q)
    sv = pg.start_vectors(q.n, count=24)
    note(f"double eigenvalues n={q.n} k={k}")
    P = K.Pencil.from_pencilgen(ctx, q)
    lam_k, x, info = P.eig(k, start_vectors=sv)
    assert info["si_block"] > 1 and info["si_block"] == info["nu_upper"] - info["nu_lower"]
    assert info["k_validated"] == k
    assert abs(lam_k - lam[k - 1]) <= 1e-10 * nA
    A, B = q.A(), q.B()
    assert np.linalg.norm(A @ x - lam_k * (B @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    assert abs(x @ (B @ x) - 1.0) < 1e-10
    for s, v in zip(info["sigmas"], info["nus"]):
        assert v == od.nu(lam, s)
    ref = o3.kth_eig(q, k)
    assert ref.si_block == info["si_block"]
    assert abs(lam_k - ref.lam) <= 1e-10 * nA


def test_double_eigenvalue_single_vector_fails(K, ctx, doubled):
    q, lam = doubled
    note("double eigenvalues, Alg. 3 only")
    P = K.Pencil.from_pencilgen(ctx, q)
    with pytest.raises(K.KthError) as e:
        P.eig(q.n // 2, start_vectors=pg.start_vectors(q.n), si_block=1, max_lanczos=120)
    assert e.value.status in (K.KTH_ECLUSTER, K.KTH_ENOCONV)


def test_block_on_simple_eigenvalues(K, ctx):
    p = pg.workload("tiny")
    lam = od.eigvals(p)
    nA = od.norm_inf(p)
    note("block SI Lanczos, simple eigenvalues")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(p.n, count=12)
    l1, x1, i1 = P.eig(p.k, start_vectors=sv, si_block=1)
    for b in (2, 5):
        lb, xb, ib = P.eig(p.k, start_vectors=sv, si_block=b)
        assert ib["si_block"] == b and ib["k_validated"] == p.k
        assert abs(lb - lam[p.k - 1]) <= 1e-10 * nA and abs(lb - l1) <= 1e-12 * nA
        assert np.linalg.norm(xb - x1) <= 1e-8 * np.linalg.norm(x1)
        assert ib["si_steps"] < i1["si_steps"]
