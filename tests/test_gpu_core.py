"""GPU parity of the hot path against the oracle (through the C ABI).

* nu(sigma) from the GPU LDL^T equals the oracle's count bit for bit;
* solves with a kept factor: backward error;
* the three-stage eigenpair on the n = 2048 tight-binding pencil vs the dense oracle.
"""
import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from oracle import sparse as osp
from tests.closed_form import chain_eigs, fem_eigs
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    note("context")
    return K.Context(0)


def _pencils():
    return [
        ("chain", pg.chain(300, 0.2, -1.0), chain_eigs(300, 0.2, -1.0)),
        ("fem", pg.fem_tensor((7, 8, 9)), fem_eigs((7, 8, 9))),
        ("blockdiag", pg.block_diag_perm((30, 17, 41, 5, 64), seed=2), None),
        ("tb2", pg.tb_supercell((2, 2, 2), seed=1), None),
        ("tb4", pg.tb_supercell((4, 4, 4), seed=0), None),
        ("tb6x5x4", pg.tb_supercell((6, 5, 4), seed=3), None),
    ]


@pytest.mark.parametrize("idx", range(6))
def test_inertia_matches_oracle(K, ctx, idx):
    name, p, ref = _pencils()[idx]
    if ref is None:
        ref, _ = od.eig(p)
    note(f"inertia {name} n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p, check_symmetry=True)
    rng = np.random.default_rng(idx)
    sig = rng.uniform(ref[0] - 0.1 * abs(ref[0]) - 0.1, ref[-1] + 0.1 * abs(ref[-1]) + 0.1, 40)
    spread = ref[-1] - ref[0]
    for s in sig:
        if np.min(np.abs(ref - s)) < 1e-9 * spread:
            continue
        nu, nz = P.inertia(s)
        assert nz == 0
        assert nu == int(np.sum(ref < s)), (name, s)
    # the sparse oracle on the same shifts (independent factorization)
    for s in sig[:8]:
        if np.min(np.abs(ref - s)) < 1e-9 * spread:
            continue
        assert P.nu(s) == osp.nu(p, s)


def test_factor_solve_backward_error(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    note("factor+solve tb4")
    P = K.Pencil.from_pencilgen(ctx, p)
    sigma = -3.0
    F = P.factor(sigma)
    neg, zero, pos = F.inertia()
    assert neg + zero + pos == p.n and zero == 0
    rng = np.random.default_rng(5)
    b = rng.normal(size=(p.n, 3))
    x = F.solve(b)
    C = p.A() - sigma * p.B()
    for q in range(3):
        r = C @ x[:, q] - b[:, q]
        berr = np.linalg.norm(r) / (od.norm_inf(p) * np.linalg.norm(x[:, q]) + np.linalg.norm(b[:, q]))
        assert berr < 1e-12, berr


def test_three_stage_tiny(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    k = p.n // 2
    lam_ref, x_ref = od.kth(p, k)
    note("kth_eig tb4")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(p.n)
    lam, x, info = P.eig(k, start_vectors=sv)
    nA = od.norm_inf(p)
    assert info["k_validated"] == k
    assert abs(lam - lam_ref) <= 1e-10 * nA
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
    A, B = p.A(), p.B()
    assert np.linalg.norm(A @ x - lam * (B @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    assert abs(x @ (B @ x) - 1) < 1e-10
    # every shift the GPU visited has the oracle's count
    lam_all, _ = od.eig(p)
    for s, nu in zip(info["sigmas"], info["nus"]):
        assert nu == od.nu(lam_all, s)
