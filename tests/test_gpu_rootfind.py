"""The interpolating stage 2 (kth_opts.root_finder = 1) on the GPU against the
oracle's run of the same algorithm.

* tiny workload: the library visits the oracle's shifts to rounding (same start
  vectors, the same interpolation arithmetic; the stage-1 Ritz values may differ
  in their last bits), with the dense counts, the oracle's counts and number of
  steps, and lambda_k of the dense definition;
* a tensor-FEM pencil: every count equals the closed form;
* the option is refused together with multisection.
"""
import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from oracle import three_stage as o3
from tests.closed_form import fem_eigs
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


def test_interp_replays_oracle_tiny(K, ctx):
    p = pg.workload("tiny")
    ref = o3.kth_eig(p, root_finder="interp")
    lam_d = od.eigvals(p)
    note("root_finder=1 tiny")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n), root_finder=1)
    assert info["k_validated"] == p.k
    assert abs(lam - lam_d[p.k - 1]) <= 1e-10 * od.norm_inf(p)
    # every count is the dense count; the shifts follow the oracle's to rounding
    # (stage-1 Ritz values differ in the last bits with the reduction order), with
    # the same counts, the same number of steps and the same final counts
    for s, v in zip(info["sigmas"], info["nus"]):
        assert v == od.nu(lam_d, s)
    assert len(info["sigmas"]) == len(ref.sigmas)
    nA = od.norm_inf(p)
    for a, b in zip(info["sigmas"], ref.sigmas):
        assert abs(a - b) <= 1e-12 * nA
    assert info["nus"] == ref.nus
    assert (info["nu_lower"], info["nu_upper"]) == (ref.nu_lower, ref.nu_upper)
    assert info["bisection_steps"] == ref.bisection_steps
    base = P.eig(p.k, start_vectors=pg.start_vectors(p.n))[2]
    assert info["n_factorizations"] < base["n_factorizations"]


def test_interp_fem_closed_form(K, ctx):
    N, w = (11, 12, 13), (1.0, 1.3, 0.7)
    p = pg.fem_tensor(N, w)
    ref = fem_eigs(N, w)
    note(f"root_finder=1 fem n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    for k in (p.n // 5, p.n // 2, (4 * p.n) // 5):
        lam, _, info = P.eig(k, start_vectors=pg.start_vectors(p.n), root_finder=1)
        assert info["k_validated"] == k
        assert abs(lam - ref[k - 1]) <= 1e-10 * od.norm_inf(p)
        for s, v in zip(info["sigmas"], info["nus"]):
            assert v == int(np.sum(ref < s))
        assert info["nu_upper"] - info["nu_lower"] <= 20


@pytest.mark.parametrize("rf", [0, 1])
def test_automatic_m_max(K, ctx, rf):
    p = pg.workload("tiny")
    lam_d = od.eigvals(p)
    note(f"m_max=0 root_finder={rf}")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n), root_finder=rf, m_max=0)
    assert info["k_validated"] == p.k
    assert abs(lam - lam_d[p.k - 1]) <= 1e-10 * od.norm_inf(p)
    m = info["m_max_used"]
    assert (m == 2) if rf == 1 else (2 <= m <= 20)
    assert info["nu_upper"] - info["nu_lower"] <= m
    for s, v in zip(info["sigmas"], info["nus"]):
        assert v == od.nu(lam_d, s)
    # the oracle's stage 2 with the same stopping count reaches the same counts
    ref = o3.kth_eig(p, m_max=m, root_finder="interp" if rf == 1 else "bisection")
    assert (ref.nu_lower, ref.nu_upper) == (info["nu_lower"], info["nu_upper"])


def test_interp_rejects_multisection(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=1)
    note("root_finder=1 with multisection")
    P = K.Pencil.from_pencilgen(ctx, p)
    with pytest.raises(K.KthError) as e:
        P.eig(p.k, root_finder=1, multisection=4)
    assert e.value.status == K.KTH_EINVAL
