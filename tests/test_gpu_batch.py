"""Batched multisection and batched pencils on the GPU.

* 64 shifts of the n = 131072 pencil factored together: every count equals the
  one-at-a-time count and, at the oracle's stored shifts, the oracle's count;
* multisection inside kth_eig gives the same validated eigenpair;
* a batch of uneven open-cluster pencils through kth_eig_batch against the
  dense oracle.
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


def test_eig_batch_uneven_pencils(K, ctx):
    pens = pg.uneven_batch(count=256, seed=0)
    pick = [q for q in range(len(pens)) if pens[q].n <= 2400][:6]
    sel = [pens[q] for q in pick]
    note(f"eig batch {[p.n for p in sel]}")
    Ps = [K.Pencil.from_pencilgen(ctx, p) for p in sel]
    res = K.eig_batch(ctx, Ps, [p.k for p in sel])
    for p, (st, lam, x, info) in zip(sel, res):
        assert st == K.KTH_OK
        lam_ref, _ = od.kth(p, p.k)
        assert info["k_validated"] == p.k
        assert abs(lam - lam_ref) <= 1e-10 * od.norm_inf(p)


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
