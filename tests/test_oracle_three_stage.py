"""Pins of the oracle's three-stage driver (Alg. 2 -> Alg. 1' -> Alg. 3).

Checked against values that do not come from the driver itself: the dense
definition of lambda_k, closed-form spectra, Prop. 1, Prop. 2, eq. (res2),
Prop. 3, the bisection step count of Alg. 1, and the printed footnote case of
Section 4.3.2.
"""
import math

import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from oracle import sparse as osp
from oracle import three_stage as o3
from tests.closed_form import fem_eigs


@pytest.fixture(scope="module")
def tiny():
    p = pg.tb_supercell((4, 4, 4), seed=0)
    lam, X = od.eig(p)
    return p, lam, X


def test_three_stage_tiny_matches_dense(tiny):
    p, lam, X = tiny
    k = p.n // 2
    r = o3.kth_eig(p, k)
    nA = od.norm_inf(p)
    assert r.k_validated == k
    assert abs(r.lam - lam[k - 1]) <= 1e-10 * nA
    x = od.sign_fix(X[:, k - 1])
    assert np.linalg.norm(r.x - x) / np.linalg.norm(x) < 1e-9
    assert r.rel_residual < 1e-9 * nA
    # interval bookkeeping: nu values are the dense counts
    assert r.nu_lower == od.nu(lam, r.sigma_lower) and r.nu_upper == od.nu(lam, r.sigma_upper)
    assert r.nu_upper - r.nu_lower <= 20
    assert r.nu_lower < k <= r.nu_upper
    for s, nu in zip(r.sigmas, r.nus):
        assert nu == od.nu(lam, s)
    # Section 4.3.1: two stage-1 iterations are the minimum to validate an interval
    assert r.stage1_steps >= 2


def test_three_stage_fem_closed_form():
    N, w = (7, 8, 9), (1.0, 1.31, 1.73)
    ref = fem_eigs(N, w)
    p = pg.fem_tensor(N, w)
    # choose a k whose eigenvalue is simple and well separated
    gaps = np.minimum(np.diff(ref)[:-1], np.diff(ref)[1:]) / ref[-1]
    cands = [k for k in range(p.n // 3, 2 * p.n // 3) if gaps[k - 2] > 1e-3]
    k = cands[len(cands) // 2]
    r = o3.kth_eig(p, k)
    assert abs(r.lam - ref[k - 1]) <= 1e-10 * od.norm_inf(p)


def test_stage3_propositions(tiny):
    """Prop. 1 (collinearity iff v~_{j+1} = 0), Prop. 2 (B-cosines), eq. (res2)
    (residual), Prop. 3 (each bound holds a true eigenvalue)."""
    p, lam, X = tiny
    A, B = p.A(), p.B()
    k = p.n // 2
    sl, su = 0.5 * (lam[k - 8] + lam[k - 9]), 0.5 * (lam[k + 4] + lam[k + 5])
    nl, nu_ = od.nu(lam, sl), od.nu(lam, su)
    rec = []
    v0 = pg.start_vectors(p.n)[1]
    o3.stage3(p, k, sl, su, nl, nu_, A, B, v0, trace=rec.append)
    assert rec
    nA = od.norm_inf(p)
    for t in rec[::3]:
        sig, th, Y, order = t["sigma"], t["theta"], t["Y"], t["order"]
        for c, i in enumerate(order):
            x2 = t["X"][:, c]
            li = sig + 1.0 / th[i]
            # eq. (res2): (A - lambda_i B) x_{i,2} = -v~_{j+1} s_i
            r = A @ x2 - li * (B @ x2)
            assert np.linalg.norm(r + t["vtnext"] * t["s"][c]) <= 1e-9 * np.linalg.norm(r) + 1e-11 * nA * np.linalg.norm(x2)
            # Prop. 3: an eigenvalue within eta_i (tiny slack for rounding)
            assert np.min(np.abs(lam - li)) <= t["eta"][c] * (1 + 1e-6) + 1e-12 * nA
        # Prop. 2 on the first two pairs
        if len(order) >= 2:
            xa, xb = t["X"][:, 0], t["X"][:, 1]
            lhs = abs(xa @ (B @ xb)) / math.sqrt((xa @ (B @ xa)) * (xb @ (B @ xb)))
            sa, sb = abs(t["s"][0]), abs(t["s"][1])
            rhs = sa / math.sqrt(1 + sa * sa) * sb / math.sqrt(1 + sb * sb)
            assert abs(lhs - rhs) <= 1e-8 * max(rhs, 1e-6) + 1e-12


def test_prop1_collinear_iff_breakdown():
    """Start the SI Lanczos inside the span of 3 exact eigenvectors: after 3
    steps v~_4 = 0 and x_{i,2} = theta_i x_{i,1}; before that they differ."""
    p = pg.tb_supercell((2, 2, 2), seed=3)
    lam, X = od.eig(p)
    A, B = p.A(), p.B()
    k = p.n // 2
    idx = [k - 2, k - 1, k]
    v0 = X[:, idx] @ np.array([0.7, -0.5, 0.4])
    sl, su = 0.5 * (lam[k - 4] + lam[k - 3]), 0.5 * (lam[k + 1] + lam[k + 2])
    nl, nu_ = od.nu(lam, sl), od.nu(lam, su)
    rec = []
    with pytest.raises(o3.NoConvergence):
        # m = 5 eigenvalues in the interval but the Krylov space has dimension 3
        o3.stage3(p, k, sl, su, nl, nu_, A, B, v0, trace=rec.append, max_iter=3)
    # run the raw recurrence by hand through the oracle's pieces for j = 1..3
    F = osp.Factor(p, 0.5 * (sl + su))
    v = v0 / math.sqrt(v0 @ (B @ v0))
    V, Vt, al, be = [v], [B @ v], [], []
    for j in range(1, 4):
        w = F.solve(Vt[-1])
        Bw = B @ w
        Vm, Vtm = np.array(V).T, np.array(Vt).T
        for _ in range(2):
            h = Vtm.T @ w
            if _ == 0:
                al.append(h[-1])
            w -= Vm @ h
            Bw -= Vtm @ h
        beta = math.sqrt(max(w @ Bw, 0.0))
        T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
        th, Y = np.linalg.eigh(T)
        x1 = Vm @ Y[:, -1]                             # x_{i,1} = B^{-1} V~ y
        x2 = F.solve(Vtm @ Y[:, -1])                   # x_{i,2} = (A - sigma B)^{-1} V~ y
        cos = abs(x1 @ x2) / (np.linalg.norm(x1) * np.linalg.norm(x2))
        if j < 3:
            assert beta > 1e-8 and 1 - cos > 1e-10
        else:
            assert beta < 1e-8 * abs(al[0]) + 1e-10 and 1 - cos < 1e-12
        be.append(beta)
        V.append(w / beta if beta > 1e-300 else w)
        Vt.append(Bw / beta if beta > 1e-300 else Bw)


def test_alg1_step_count_and_accuracy(tiny):
    p, lam, _ = tiny
    k = p.n // 2
    P = osp.prepare(p)
    sl, su = lam[0] - 0.1, lam[-1] + 0.1
    tau = 1e-6
    est, a, b, steps = o3.alg1_bisection(k, sl, su, lambda s: od.nu(lam, s), tau=tau)
    assert steps == math.ceil(math.log2((su - sl) / tau))
    assert abs(est - lam[k - 1]) < tau / 2
    # the same with the sparse oracle's inertia, fewer steps for spot checking
    est2, *_ = o3.alg1_bisection(k, sl, su, lambda s: osp.nu(P, s), tau=1e-3)
    assert abs(est2 - lam[k - 1]) < 0.5e-3


def test_straightforward_bisection_footnote_count():
    """Section 4.3.2: relative-width bisection from the APF4686 initial interval
    [-0.777, 0.475) (Table 4) to the 1e-14 criterion needs 47-49 steps (printed
    range).  Model nu by a step function at the printed lambda_k (Table 2)."""
    lam_k = -0.4258775547956963
    est, a, b, steps = o3.alg1_bisection(1, -0.777, 0.475, lambda s: int(s > lam_k),
                                         rel_tau=1e-14)
    assert 47 <= steps <= 49
    assert abs(est - lam_k) < 1e-14


def _diag_count(eigs):
    eigs = np.sort(np.asarray(eigs, dtype=float))
    return lambda s: int(np.searchsorted(eigs, s, side="left"))


def test_interp_stage2_linear_count_lands_in_two_steps():
    # eigenvalues 1..n: the count is linear between the bracket ends up to its
    # unit steps, so each interpolated shift lands within one of its target count:
    # the first brings the lower end to k - m/2, the second the upper to k + m/2 - 1
    n, k, m = 1000, 400, 20
    nu_of = _diag_count(np.arange(1, n + 1))
    log = []
    sl, su, nl, nu_, steps = o3.stage2_interp(k, 0.5, n + 0.5, 0, n, nu_of, log, m_max=m)
    assert steps == 2
    assert k - m // 2 - 1 <= nl < k <= nu_ <= k + m // 2
    assert nu_ - nl <= m
    # the same bracket by bisection takes ceil(log2(n / m)) steps at least
    log2 = []
    assert o3.stage2(k, 0.5, n + 0.5, 0, n, nu_of, log2, m_max=m)[4] >= math.ceil(math.log2(n / m))


def test_interp_stage2_cluster_falls_back_to_bisection():
    # 1000 eigenvalues piled into [50, 50.001] among 1..100: the linear model is
    # badly wrong, the safeguard's midpoint steps still isolate k
    eigs = np.concatenate([np.arange(1.0, 101.0), 50.0 + np.linspace(1e-4, 1e-3, 1000)])
    nu_of = _diag_count(eigs)
    lam = np.sort(eigs)
    for k in (30, 300, 1060):
        log = []
        sl, su, nl, nu_, steps = o3.stage2_interp(k, 0.5, 100.5, 0, eigs.size, nu_of, log)
        assert nl == nu_of(sl) and nu_ == nu_of(su)
        assert nl < k <= nu_ and nu_ - nl <= 20
        assert sl < lam[k - 1] < su
        log2 = []
        assert steps <= 3 * o3.stage2(k, 0.5, 100.5, 0, eigs.size, nu_of, log2)[4]


@pytest.mark.parametrize("which", ["tiny", "fem"])
def test_three_stage_interp_matches_dense(which):
    if which == "tiny":
        p = pg.tb_supercell((4, 4, 4), seed=0)
        lam = od.eigvals(p)
    else:
        N, w = (9, 10, 11), (1.0, 1.4, 0.8)
        p = pg.fem_tensor(N, w)
        lam = fem_eigs(N, w)
    k = p.k
    nA = od.norm_inf(p)
    rb = o3.kth_eig(p, k)
    ri = o3.kth_eig(p, k, root_finder="interp")
    assert ri.k_validated == k
    assert abs(ri.lam - lam[k - 1]) <= 1e-10 * nA
    assert ri.nu_lower == od.nu(lam, ri.sigma_lower) and ri.nu_upper == od.nu(lam, ri.sigma_upper)
    assert ri.nu_lower < k <= ri.nu_upper and ri.nu_upper - ri.nu_lower <= 20
    for s, v in zip(ri.sigmas, ri.nus):
        assert v == od.nu(lam, s)
    assert ri.bisection_steps < rb.bisection_steps


@pytest.fixture(scope="module")
def doubled():
    q = pg.doubled(pg.tb_cluster(200, seed=4), seed=None)
    return q, od.eigvals(q)


def test_block_si_lanczos_double_eigenvalues(doubled):
    # every eigenvalue is exactly double: Alg. 3 with one start vector sees one
    # copy of each, so it cannot validate m bounds; the block method does
    q, lam = doubled
    nA = od.norm_inf(q)
    for k in (q.n // 2, q.n // 2 + 1, 241):
        r = o3.kth_eig(q, k)
        assert r.si_block > 1 and r.si_block == r.nu_upper - r.nu_lower
        assert r.k_validated == k
        assert abs(r.lam - lam[k - 1]) <= 1e-10 * nA
        assert r.rel_residual <= 1e-9 * nA
        assert abs(r.x @ (q.B() @ r.x) - 1.0) < 1e-12
    with pytest.raises(o3.NoConvergence):
        o3.kth_eig(q, q.n // 2, si_block=1, max_iter=120)


def test_block_si_lanczos_matches_single_vector(tiny):
    p, lam, X = tiny
    k = p.n // 2
    nA = od.norm_inf(p)
    r1 = o3.kth_eig(p, k, si_block=1)
    for b in (2, 5):
        rb = o3.kth_eig(p, k, si_block=b)
        assert rb.si_block == b and rb.k_validated == k
        assert abs(rb.lam - lam[k - 1]) <= 1e-10 * nA
        assert abs(rb.lam - r1.lam) <= 1e-12 * nA
        assert rb.si_steps < r1.si_steps        # p vectors per step
        x = od.sign_fix(X[:, k - 1])
        assert np.linalg.norm(od.sign_fix(rb.x / np.sqrt(rb.x @ (p.B() @ rb.x))) - x) < 1e-8


def test_block_start_columns():
    n = 50
    V = o3.block_start(n, 4)
    sv = pg.start_vectors(n)
    assert np.array_equal(V[:, 0], sv[1])
    assert np.array_equal(V[:, 1], pg.start_vectors(n, count=7)[4])
