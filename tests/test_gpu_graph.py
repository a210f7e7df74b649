"""Factorizations replayed from a captured HIP graph against kernel-by-kernel
launches (KTH_GRAPHS=0): the same counts at many shifts, replayed again and again
with other work (solves, kept factors, synchronisations) in between, and the same
three-stage result bit for bit."""
import os

import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


def _contexts(K):
    os.environ["KTH_GRAPHS"] = "0"
    try:
        eager = K.Context(0)
    finally:
        del os.environ["KTH_GRAPHS"]
    return eager, K.Context(0)


@pytest.mark.parametrize("cells", [(4, 4, 4), (8, 8, 8)])
def test_graph_replays_match_eager(cells):
    K = kth()
    ce, cg = _contexts(K)
    p = pg.tb_supercell(cells, seed=1)
    note(f"graph replays n={p.n}")
    Pe = K.Pencil.from_pencilgen(ce, p)
    Pg = K.Pencil.from_pencilgen(cg, p)
    rng = np.random.default_rng(5)
    sig = rng.uniform(-7.0, 1.0, 12)
    b = rng.normal(size=p.n)
    for rep in range(3):
        for s in sig:
            assert Pg.inertia(s) == Pe.inertia(s), (rep, s)
        # other work between the replays: a kept factor and its solves
        Fg, Fe = Pg.factor(sig[rep]), Pe.factor(sig[rep])
        assert np.array_equal(Fg.solve(b), Fe.solve(b))
        Fg.close()
        Fe.close()
    if p.n <= 4096:
        lam = od.eigvals(p)
        for s in sig:
            assert Pg.nu(s) == od.nu(lam, s)
    sv = pg.start_vectors(p.n)
    le, xe, ie = Pe.eig(p.k, start_vectors=sv, root_finder=1, m_max=0)
    for rep in range(2):    # the second call replays the kept factors' graphs
        lg, xg, ig = Pg.eig(p.k, start_vectors=sv, root_finder=1, m_max=0)
        assert lg == le and np.array_equal(xg, xe)
        assert ig["sigmas"] == ie["sigmas"] and ig["nus"] == ie["nus"]
        Pg.nu(-3.0)
