"""Stage-1 B-solves by Jacobi-preconditioned conjugate gradients
(kth_opts.b_solver = 1).

* tight-binding pencils have a strictly diagonally dominant overlap matrix B
  with a positive diagonal (positive definite by Gershgorin's theorem): the
  library skips the factor of B, lambda_k is the dense definition's, every
  count is the dense count, and the run has one factorization fewer than with
  the factor of B;
* the mass matrix of the tensor-FEM pencil is not diagonally dominant: the
  option falls back to the factor and reaches the closed form;
* values outside {0, 1} are refused.
"""
import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from tests.closed_form import fem_eigs
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


@pytest.mark.parametrize("rf", [0, 1])
def test_cg_b_solve_tiny(K, ctx, rf):
    p = pg.workload("tiny")
    lam_d = od.eigvals(p)
    nA = od.norm_inf(p)
    note(f"b_solver=1 tiny root_finder={rf}")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(p.n)
    lam, x, info = P.eig(p.k, start_vectors=sv, root_finder=rf, b_solver=1)
    assert info["b_cg_iterations"] > 0
    assert info["k_validated"] == p.k
    assert abs(lam - lam_d[p.k - 1]) <= 1e-10 * nA
    for s, v in zip(info["sigmas"], info["nus"]):
        assert v == od.nu(lam_d, s)
    A, B = p.A(), p.B()
    assert np.linalg.norm(A @ x - lam * (B @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    assert abs(x @ (B @ x) - 1.0) < 1e-10
    lf, xf, inf_ = P.eig(p.k, start_vectors=sv, root_finder=rf, b_solver=0)
    assert inf_["b_cg_iterations"] == 0
    assert info["n_factorizations"] == inf_["n_factorizations"] - 1
    # the same Krylov space to the CG tolerance: the same stage-1 run
    assert info["stage1_steps"] == inf_["stage1_steps"]
    assert abs(lam - lf) <= 1e-12 * nA


def test_cg_b_solve_not_dominant_falls_back(K, ctx):
    N, w = (9, 10, 11), (1.0, 1.3, 0.7)
    p = pg.fem_tensor(N, w)
    ref = fem_eigs(N, w)
    k = p.n // 3
    note(f"b_solver=1 fem n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, _, info = P.eig(k, start_vectors=pg.start_vectors(p.n), b_solver=1)
    assert info["b_cg_iterations"] == 0
    assert info["k_validated"] == k
    assert abs(lam - ref[k - 1]) <= 1e-10 * od.norm_inf(p)
    base = P.eig(k, start_vectors=pg.start_vectors(p.n), b_solver=0)[2]
    assert info["n_factorizations"] == base["n_factorizations"]


def test_b_solver_validation(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=1)
    note("b_solver=2")
    P = K.Pencil.from_pencilgen(ctx, p)
    with pytest.raises(K.KthError) as e:
        P.eig(p.k, b_solver=2)
    assert e.value.status == K.KTH_EINVAL
