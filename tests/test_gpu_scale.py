"""GPU parity at the workloads' full sizes, against stored oracle values and
closed forms (see tests/golden/make_golden.py: every stored value comes from
the oracle alone).

* nu(sigma) of the n = 131072 and n = 524288 tight-binding pencils equals the
  plain-C oracle's count at fixed shifts, bit for bit;
* kth_eig on n = 131072: validated index, lambda_k against the oracle's own
  three-stage run, residual, and an inertia bracket of the returned value;
* a large tensor-FEM pencil: nu equals the closed-form count.
"""
import glob
import json
import os

import numpy as np
import pytest

import pencilgen as pg
from tests.closed_form import fem_eigs
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(pattern):
    return [json.load(open(f)) for f in sorted(glob.glob(os.path.join(GOLD, pattern)))]


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


@pytest.mark.parametrize("cfg", ["n131k", "n524k"])
def test_inertia_full_size_matches_oracle(K, ctx, cfg):
    gold = _golden(f"inertia_{cfg}_*.json")
    assert gold, f"no stored oracle counts for {cfg}"
    p = pg.workload(cfg)
    note(f"inertia {cfg} n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    for g in gold:
        assert g["n"] == p.n and g["zero"] == 0
        nu, nz = P.inertia(g["sigma"])
        assert nz == 0
        assert nu == g["nu"], (cfg, g["sigma"], nu, g["nu"])


def test_eig_n131k(K, ctx):
    p = pg.workload("n131k")
    note("kth_eig n131k")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n))
    A, B = p.A(), p.B()
    nA = float(np.add.reduceat(np.abs(p.a_val), p.rowptr[:-1]).max())
    assert info["k_validated"] == p.k
    assert info["nu_lower"] < p.k <= info["nu_upper"]
    assert np.linalg.norm(A @ x - lam * (B @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    assert abs(x @ (B @ x) - 1) < 1e-10
    # inertia bracket of the returned eigenvalue: nu(lam - d) < k <= nu(lam + d)
    d = 1e-10 * nA
    assert P.nu(lam - d) < p.k <= P.nu(lam + d)
    gold = _golden("three_stage_n131k.json")
    assert gold, "no stored oracle three-stage run for n131k"
    g = gold[0]
    assert abs(lam - g["lam"]) <= 1e-10 * nA
    # replay: the library and the oracle run the same algorithm from the same start
    # vectors, so they visit the same shifts; every shared shift has the same count
    # and the final interval is the oracle's, bit for bit
    gmap = dict(zip(g["sigmas"], g["nus"]))
    shared = [(s, v) for s, v in zip(info["sigmas"], info["nus"]) if s in gmap]
    assert all(v == gmap[s] for s, v in shared), [(s, v, gmap[s]) for s, v in shared]
    assert len(shared) == len(g["sigmas"]) == len(info["sigmas"]), (info["sigmas"], g["sigmas"])
    assert (info["sigma_lower"], info["sigma_upper"], info["nu_lower"], info["nu_upper"]) == \
        (g["sigma_lower"], g["sigma_upper"], g["nu_lower"], g["nu_upper"])


def test_fem_large_closed_form(K, ctx):
    N, w = (40, 48, 56), (1.0, 1.31, 1.73)
    p = pg.fem_tensor(N, w)
    ref = fem_eigs(N, w)
    note(f"inertia fem n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    rng = np.random.default_rng(3)
    for q in rng.integers(1, p.n - 1, 6):
        s = 0.5 * (ref[q - 1] + ref[q])
        if ref[q] - ref[q - 1] < 1e-9 * ref[-1]:
            continue
        assert P.nu(s) == q


def test_eig_n131k_interp(K, ctx):
    """The interpolating stage 2 at n = 131072 against the oracle's own run of it."""
    gold = _golden("three_stage_n131k_interp.json")
    assert gold, "no stored oracle run of the interpolating stage 2 for n131k"
    g = gold[0]
    p = pg.workload("n131k")
    note("kth_eig n131k root_finder=1")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n), root_finder=1, m_max=g.get("m_max", 20))
    nA = float(np.add.reduceat(np.abs(p.a_val), p.rowptr[:-1]).max())
    assert info["k_validated"] == p.k
    assert abs(lam - g["lam"]) <= 1e-10 * nA
    assert np.linalg.norm(p.A() @ x - lam * (p.B() @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    # the same shifts (same stage-1 Ritz values, same interpolation arithmetic) and counts
    assert info["sigmas"] == g["sigmas"] and info["nus"] == g["nus"]
    assert (info["sigma_lower"], info["sigma_upper"], info["nu_lower"], info["nu_upper"]) == \
        (g["sigma_lower"], g["sigma_upper"], g["nu_lower"], g["nu_upper"])
    assert info["bisection_steps"] == g["bisection_steps"]
