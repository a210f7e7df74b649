"""Batched multisection and batched pencils on the GPU.

* 64 shifts of the n = 131072 pencil factored together: every count equals the
  one-at-a-time count and, at the oracle's stored shifts, the oracle's count;
* multisection inside kth_eig gives the same validated eigenpair;
* all 256 uneven open-cluster pencils through kth_eig_batch against the
  dense oracle's stored values.
"""
import glob
import json
import os
import time

import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


def test_inertia_batch_64_shifts_n131k(K, ctx):
    p = pg.workload("n131k")
    gold = [json.load(open(f)) for f in sorted(glob.glob(os.path.join(GOLD, "inertia_n131k_*.json")))]
    sig = np.concatenate([np.linspace(-3.6, -2.4, 64 - len(gold)), [g["sigma"] for g in gold]])
    note("inertia batch 64 n131k")
    P = K.Pencil.from_pencilgen(ctx, p)
    P.inertia_batch(sig[:4])                      # allocate the batch storage
    t0 = time.perf_counter()
    nb = P.inertia_batch(sig)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = [P.nu(s) for s in sig]
    t_single = time.perf_counter() - t0
    print(f"64 shifts: batched {t_batch:.3f} s, one at a time {t_single:.3f} s")
    assert nb.tolist() == single
    for g in gold:
        assert nb[list(sig).index(g["sigma"])] == g["nu"]
    assert all(np.diff(nb[: 64 - len(gold)]) >= 0)


def test_multisection_eig(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    k = p.n // 2
    lam_ref, _ = od.kth(p, k)
    note("multisection kth_eig")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(p.n)
    base = P.eig(k, start_vectors=sv)
    for ms in (3, 8):
        lam, x, info = P.eig(k, start_vectors=sv, multisection=ms)
        assert info["k_validated"] == k
        assert abs(lam - lam_ref) <= 1e-10 * od.norm_inf(p)
        assert info["bisection_steps"] < base[2]["bisection_steps"]


def test_eig_batch_256_uneven_pencils(K, ctx):
    """All 256 pencils of the uneven batch (n in [500, 8000]) in one kth_eig_batch
    call, each against the dense oracle's lambda_k stored in
    tests/golden/batch_dense_256.json (written by make_golden.py from oracle.dense)."""
    gold = json.load(open(os.path.join(GOLD, "batch_dense_256.json")))["pencils"]
    pens = pg.uneven_batch(count=256, seed=0)
    assert len(gold) == len(pens)
    note(f"eig batch of {len(pens)} pencils, n {min(p.n for p in pens)}..{max(p.n for p in pens)}")
    Ps = [K.Pencil.from_pencilgen(ctx, p) for p in pens]
    t0 = time.perf_counter()
    res = K.eig_batch(ctx, Ps, [p.k for p in pens])
    print(f"256 pencils: {time.perf_counter() - t0:.2f} s")
    for p, g, (st, lam, x, info) in zip(pens, gold, res):
        assert (g["n"], g["k"]) == (p.n, p.k)
        assert st == K.KTH_OK, (g["i"], st)
        assert info["k_validated"] == p.k
        assert abs(lam - g["lam"]) <= 1e-10 * g["norm_a_inf"], (g["i"], lam, g["lam"])
        r = p.A() @ x - lam * (p.B() @ x)
        assert np.linalg.norm(r) / (g["norm_a_inf"] * np.linalg.norm(x)) <= 1e-9
        assert abs(x @ (p.B() @ x) - 1.0) < 1e-10
    for P_ in Ps:
        P_.close()


def test_eig_batch_workers_match_sequential(K, ctx):
    # concurrent workers give the same results as one pencil after another, and a
    # bad k fails only its own pencil
    ps = pg.uneven_batch(12, seed=3, n_lo=300, n_hi=1500)
    note(f"eig batch workers vs sequential, n {[p.n for p in ps]}")
    Ps = [K.Pencil.from_pencilgen(ctx, p) for p in ps]
    ks = [p.k for p in ps]
    ks[5] = ps[5].n + 1                      # invalid
    seq = K.eig_batch(ctx, Ps, ks, batch_workers=1)
    par = K.eig_batch(ctx, Ps, ks, batch_workers=6)
    for i, (a, b) in enumerate(zip(seq, par)):
        if i == 5:
            assert a[0] == b[0] == K.KTH_EINVAL
            continue
        assert a[0] == b[0] == K.KTH_OK
        assert a[1] == b[1] and np.array_equal(a[2], b[2])
        assert a[3]["k_validated"] == b[3]["k_validated"] == ks[i]
        assert a[3]["sigmas"] == b[3]["sigmas"]
