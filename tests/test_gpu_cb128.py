"""Contribution blocks on 128 x 128 tiles (k_gemm_cb128) against 64 x 64 tiles
(k_gemm_lt): both give every entry the same products in the same order, so the
factors agree bit for bit.  KTH_CB128_MIN_NU, read when a pencil is created,
moves the size threshold: 1 puts every contribution block (ragged ones too) on
128-tiles, a huge value none.  Checked: the counts at many shifts, the factor
statistics, and a solve with a kept factor, all exactly equal."""
import os

import numpy as np
import pytest

import pencilgen as pg
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


def _pencil(K, ctx, p, min_nu):
    old = os.environ.get("KTH_CB128_MIN_NU")
    if min_nu is None:
        os.environ.pop("KTH_CB128_MIN_NU", None)
    else:
        os.environ["KTH_CB128_MIN_NU"] = str(min_nu)
    try:
        return K.Pencil.from_pencilgen(ctx, p)
    finally:
        if old is None:
            os.environ.pop("KTH_CB128_MIN_NU", None)
        else:
            os.environ["KTH_CB128_MIN_NU"] = old


@pytest.mark.parametrize("cells", [(4, 4, 4), (8, 8, 8), (12, 12, 8)])
def test_cb128_bit_identical(cells):
    K = kth()
    ctx = K.Context(0)
    p = pg.tb_supercell(cells, seed=1)
    note(f"cb128 n={p.n}")
    ref = _pencil(K, ctx, p, 10**9)
    rng = np.random.default_rng(11)
    sig = rng.uniform(-7.0, 1.0, 6)
    b = rng.normal(size=p.n)
    base = {}
    for s in sig:
        f = ref.factor(float(s))
        base[s] = (f.inertia(), f.stats(), f.solve(b, refine=False))
        f.close()
    for min_nu in (None, 1):
        P = _pencil(K, ctx, p, min_nu)
        for s in sig:
            f = P.factor(float(s))
            inert, st, x = f.inertia(), f.stats(), f.solve(b, refine=False)
            assert inert == base[s][0], (min_nu, s)
            assert st == base[s][1], (min_nu, s)
            assert np.array_equal(x, base[s][2]), (min_nu, s)
