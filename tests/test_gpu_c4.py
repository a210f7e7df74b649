"""lambda_k of the n = 524288 tight-binding pencil (k = n/2) against the oracle's
own run (tests/golden/kth_oracle_n524k.json, written by make_golden.py's
kth_oracle job from oracle/ alone: inertia by the oracle's sparse LDL^T at every
shift, its stage 3 for lambda, and a bracket certificate).

* every count the oracle took is the library's count at the same shift;
* the oracle's certificate holds: nu(lam - eps) < k <= nu(lam + eps), eps =
  1e-11 ||A||_inf, so its lambda_k is certified by Sylvester's law alone;
* the library's lambda_k -- plain FP64 and FP32 + refinement, bisection and the
  interpolating stage 2 -- lies within delta - eps of the oracle's (delta =
  1e-10 ||A||_inf), so within delta of the certified lambda_k, with k validated.
"""
import json
import os

import pytest

import pencilgen as pg
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kth_oracle_n524k.json")


@pytest.fixture(scope="module")
def setup():
    K = kth()
    ctx = K.Context(0)
    p = pg.workload("n524k")
    note(f"n524k pencil n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    return K, p, P, json.load(open(GOLD))


def test_oracle_counts(setup):
    K, p, P, g = setup
    assert g["phase"] == "done"
    for sigma, nu, zero in g["counts"]:
        note(f"n524k nu({sigma!r})")
        assert P.inertia(sigma) == (nu, zero), sigma


def test_oracle_certificate(setup):
    K, p, P, g = setup
    c = g["certificate"]
    assert c["holds"]
    assert c["nu_minus"] < p.k <= c["nu_plus"]
    # the certified ends are lam -+ eps (up to the rounding of a double near lam)
    assert abs(c["eps"] - 1e-11 * g["norm_a_inf"]) <= 1e-24
    assert abs((g["lam"] - c["eps"]) - c["sigma_minus"]) <= 4e-16 * abs(g["lam"])
    assert abs((g["lam"] + c["eps"]) - c["sigma_plus"]) <= 4e-16 * abs(g["lam"])


@pytest.mark.parametrize("rf,prec", [(0, "fp64"), (1, "fp64"), (1, "fp32_ir")])
def test_lambda_within_delta(setup, rf, prec):
    K, p, P, g = setup
    lam_hat = g["lam"]
    dlt = 1e-10 * g["norm_a_inf"] - g["certificate"]["eps"]
    note(f"n524k kth_eig root_finder={rf} {prec}")
    kw = dict(start_vectors=pg.start_vectors(p.n), root_finder=rf, m_max=0 if rf else 20)
    if prec == "fp32_ir":
        kw["si_precision"] = K.KTH_FP32_IR
    lam, _, info = P.eig(p.k, want_x=False, **kw)
    assert info["k_validated"] == p.k
    assert abs(lam - lam_hat) <= dlt, (lam, lam_hat)
