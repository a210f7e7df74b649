"""GPU checks of the FP32 shift-and-invert factor with FP64 iterative refinement:
refined solves reach FP64 backward error and agree with the FP64 factor; a shift
on an eigenvalue makes the refinement stall and report it (never silently); the
three-stage algorithm with the FP32 factor returns the FP64 / oracle eigenpair,
and falls back to an FP64 factor when the refinement stalls."""
import numpy as np
import pytest

import pencilgen as pg
from oracle import dense as od
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    return kth()


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


def _berr(M, x, b):
    """Normwise backward error ||b - M x||_inf / (||M||_inf ||x||_inf + ||b||_inf)."""
    r = b - M @ x
    nM = abs(M).sum(axis=1).max()
    return np.abs(r).max() / (nM * np.abs(x).max() + np.abs(b).max())


def test_fp32_factor_refined_solve(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=3)
    lam, _ = od.eig(p)
    i = p.n // 3
    sigma = 0.5 * (lam[i] + lam[i + 1])          # between two eigenvalues
    M = (p.A() - sigma * p.B()).tocsr()
    Md = M.toarray()
    kappa = np.linalg.norm(Md, np.inf) * np.linalg.norm(np.linalg.inv(Md), np.inf)
    note(f"fp32 factor solve n={p.n} sigma={sigma!r} kappa_inf={kappa:.3e}")
    P = K.Pencil.from_pencilgen(ctx, p)
    F32 = P.factor(sigma, K.KTH_FP32_IR)
    F64 = P.factor(sigma, K.KTH_FP64)
    R = np.random.default_rng(5).normal(size=(p.n, 3))
    X32 = F32.solve(R)
    X64 = F64.solve(R)
    for q in range(R.shape[1]):
        b32 = _berr(M, X32[:, q], R[:, q])
        b64 = _berr(M, X64[:, q], R[:, q])
        note(f"  column {q}: berr fp32+IR {b32:.2e}, fp64 {b64:.2e}")
        assert b32 <= 2e-14
        fwd = np.abs(X32[:, q] - X64[:, q]).max() / np.abs(X64[:, q]).max()
        assert fwd <= 10 * kappa * 2e-14, (fwd, kappa)
    # a kept FP32 factor has no certified inertia
    with pytest.raises(K.KthError) as e:
        F32.inertia()
    assert e.value.status == K.KTH_ESTATE


def test_fp32_refinement_stall_is_reported(K, ctx):
    p = pg.tb_supercell((2, 2, 3), seed=4)
    lam, _ = od.eig(p)
    gaps = np.diff(lam)
    j = int(np.argmax(np.minimum(gaps[:-1], gaps[1:]))) + 1   # best isolated eigenvalue
    sigma = float(lam[j])                                       # shift on the eigenvalue
    note(f"fp32 refinement at an eigenvalue n={p.n} sigma={sigma!r}")
    P = K.Pencil.from_pencilgen(ctx, p)
    F = P.factor(sigma, K.KTH_FP32_IR)
    b = np.random.default_rng(6).normal(size=p.n)
    M = (p.A() - sigma * p.B()).tocsr()
    try:
        x = F.solve(b)
    except K.KthError as e:
        assert e.status == K.KTH_ENOCONV
    else:   # refinement that does return must have reached the target
        assert np.all(np.isfinite(x)) and _berr(M, x, b) <= 2e-14


@pytest.mark.parametrize("cells,seed", [((3, 3, 3), 0), ((4, 4, 4), 1)])
def test_eig_fp32_si_matches_fp64(K, ctx, cells, seed):
    p = pg.tb_supercell(cells, seed=seed)
    k = p.n // 2
    sv = pg.start_vectors(p.n, seed=seed)
    note(f"eig fp32 SI n={p.n} k={k}")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam64, x64, i64 = P.eig(k, start_vectors=sv)
    lam32, x32, i32 = P.eig(k, start_vectors=sv, si_precision=K.KTH_FP32_IR)
    lam_ref, _ = od.kth(p, k)
    nA = od.norm_inf(p)
    note(f"  lambda fp64 {lam64!r} fp32+IR {lam32!r} oracle {lam_ref!r}; ir_steps "
         f"{i32['ir_steps']} over {i32['si_steps']} solves, max berr {i32['ir_max_berr']:.2e}")
    assert i32["k_validated"] == k and i64["k_validated"] == k
    assert i32["si_precision"] == K.KTH_FP32_IR and i32["ir_fallback"] == 0
    assert i32["ir_steps"] >= i32["si_steps"]          # every FP32 solve needs corrections
    assert i32["ir_max_berr"] <= 1e-14
    assert i64["si_precision"] == K.KTH_FP64 and i64["ir_steps"] == 0
    assert abs(lam32 - lam64) <= 1e-10 * nA
    assert abs(lam32 - lam_ref) <= 1e-10 * nA
    assert abs(x32 @ (p.B() @ x64)) >= 1 - 1e-8        # same B-normalised vector
    r = p.A() @ x32 - lam32 * (p.B() @ x32)
    assert np.linalg.norm(r) / (nA * np.linalg.norm(x32)) <= 1e-9


def test_eig_fp32_shift_on_eigenvalue(K, ctx):
    p = pg.tb_supercell((2, 2, 3), seed=4)
    lam, _ = od.eig(p)
    gaps = np.diff(lam)
    j = int(np.argmax(np.minimum(gaps[:-1], gaps[1:]))) + 1   # 0-based, isolated
    d = 1e-9 * max(1.0, abs(lam[j]))
    assert min(gaps[j - 1], gaps[j]) > 100 * d
    sl, su = lam[j] - d, lam[j] + d      # midpoint = the eigenvalue: M nearly singular
    note(f"eig fp32 shift on eigenvalue n={p.n} k={j + 1} interval [{sl!r}, {su!r})")
    P = K.Pencil.from_pencilgen(ctx, p)
    val, x, info = P.eig(j + 1, warm_interval=[sl, su], warm_counts=[j, j + 1],
                         si_precision=K.KTH_FP32_IR, start_vectors=pg.start_vectors(p.n))
    nA = od.norm_inf(p)
    note(f"  lambda {val!r} (oracle {lam[j]!r}), fallback {info['ir_fallback']}, "
         f"final precision {info['si_precision']}, max berr {info['ir_max_berr']:.2e}")
    assert info["k_validated"] == j + 1
    assert abs(val - lam[j]) <= 1e-10 * nA
    if info["ir_fallback"]:
        assert info["si_precision"] == K.KTH_FP64
    else:   # refinement converged on every solve
        assert info["si_precision"] == K.KTH_FP32_IR and info["ir_max_berr"] <= 1e-15


def test_eig_fp32_falls_back_to_fp64(K, ctx):
    # a refinement target no FP64 residual can reach: the first solve stalls and
    # the shift-and-invert factor is redone in FP64
    p = pg.tb_supercell((3, 3, 3), seed=2)
    k = p.n // 2
    note(f"eig fp32 forced fallback n={p.n} k={k}")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(p.n)
    val, x, info = P.eig(k, si_precision=K.KTH_FP32_IR, ir_tol=1e-300, start_vectors=sv)
    val64, _, _ = P.eig(k, start_vectors=sv)
    lam_ref, _ = od.kth(p, k)
    nA = od.norm_inf(p)
    note(f"  lambda {val!r} fp64 {val64!r} oracle {lam_ref!r}; fallback {info['ir_fallback']}")
    assert info["ir_fallback"] == 1 and info["si_precision"] == K.KTH_FP64
    assert info["k_validated"] == k
    assert abs(val - lam_ref) <= 1e-10 * nA and abs(val - val64) <= 1e-10 * nA


def test_eig_fp32_n131k_golden(K, ctx):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "three_stage_n131k.json")
    g = json.load(open(path))
    p = pg.workload("n131k")
    note(f"eig fp32 SI n={p.n} k={p.k}")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(p.k, start_vectors=pg.start_vectors(p.n), si_precision=K.KTH_FP32_IR)
    nA = od.norm_inf(p)
    note(f"  lambda {lam!r} golden {g['lam']!r}; ir_steps {info['ir_steps']} over "
         f"{info['si_steps']} solves, fallback {info['ir_fallback']}")
    assert info["k_validated"] == p.k
    assert abs(lam - g["lam"]) <= 1e-10 * nA
    assert info["rel_residual_normA"] <= 1e-9


def test_fp32_unrefined_solve(K, ctx):
    # KTH_SOLVE_UNREFINED applies the FP32 factor once: FP32-level backward error,
    # which the default (refined) solve then brings to FP64 level
    p = pg.tb_supercell((3, 3, 3), seed=6)
    sigma = -20.0                                   # below the spectrum: A - sigma B is SPD
    note(f"fp32 unrefined solve n={p.n}")
    P = K.Pencil.from_pencilgen(ctx, p)
    F = P.factor(sigma, K.KTH_FP32_IR)
    M = (p.A() - sigma * p.B()).tocsr()
    b = np.random.default_rng(7).normal(size=p.n)
    x1 = F.solve(b, refine=False)
    x2 = F.solve(b)
    b1, b2 = _berr(M, x1, b), _berr(M, x2, b)
    note(f"  berr unrefined {b1:.2e}, refined {b2:.2e}")
    assert 1e-12 < b1 < 1e-4
    assert b2 <= 2e-15


def test_eig_fp32_n524k_matches_fp64(K, ctx):
    # the precision workload: n = 524288, k = n/2, inertia factorizations in FP64,
    # the shift-and-invert factor in FP32 with FP64 refinement of every solve;
    # lambda_k and the residual against the FP64 path, and the inertia bracket
    p = pg.workload("n524k")
    sv = pg.start_vectors(p.n)
    note(f"eig fp32 SI n={p.n} k={p.k}")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam64, x64, i64 = P.eig(p.k, start_vectors=sv)
    lam32, x32, i32 = P.eig(p.k, start_vectors=sv, si_precision=K.KTH_FP32_IR)
    nA = od.norm_inf(p)
    A, B = p.A(), p.B()
    res32 = np.linalg.norm(A @ x32 - lam32 * (B @ x32)) / (nA * np.linalg.norm(x32))
    res64 = np.linalg.norm(A @ x64 - lam64 * (B @ x64)) / (nA * np.linalg.norm(x64))
    note(f"  lambda fp64 {lam64!r} fp32+IR {lam32!r} (|diff| {abs(lam32 - lam64):.2e}); residual "
         f"fp32+IR {res32:.2e} fp64 {res64:.2e}; ir_steps {i32['ir_steps']} over {i32['si_steps']} solves, "
         f"max berr {i32['ir_max_berr']:.2e}, fallback {i32['ir_fallback']}")
    assert i32["k_validated"] == p.k and i64["k_validated"] == p.k
    assert i32["si_precision"] == K.KTH_FP32_IR and i32["ir_fallback"] == 0
    assert i32["ir_max_berr"] <= 1e-14
    assert abs(lam32 - lam64) <= 1e-10 * nA
    assert res32 <= 1e-9 and res64 <= 1e-9
    assert abs(x32 @ (B @ x64)) >= 1 - 1e-8            # the same B-normalised vector
    d = 1e-10 * nA
    assert P.nu(lam32 - d) < p.k <= P.nu(lam32 + d)


def test_eig_precision_switch_same_pencil(K):
    # the shift-and-invert factor of one pencil alternates FP64 / FP32 + IR: each
    # change of precision re-lays the factor out, and a launch sequence captured for
    # the other precision must not be replayed on it (the new buffers can land at
    # the old addresses -- likely in a fresh context, whose cache holds just them)
    c = K.Context(0)
    p = pg.tb_supercell((3, 3, 3), seed=0)
    k = p.n // 2
    sv = pg.start_vectors(p.n, seed=0)
    lam_ref, _ = od.kth(p, k)
    nA = od.norm_inf(p)
    P = K.Pencil.from_pencilgen(c, p)
    for prec in (K.KTH_FP64, K.KTH_FP32_IR, K.KTH_FP64, K.KTH_FP32_IR):
        lam, x, info = P.eig(k, start_vectors=sv, si_precision=prec)
        note(f"precision switch: si_precision {prec} -> lambda {lam!r}, fallback "
             f"{info['ir_fallback']}, ir_steps {info['ir_steps']}")
        assert info["k_validated"] == k
        assert info["si_precision"] == prec and info["ir_fallback"] == 0
        assert abs(lam - lam_ref) <= 1e-10 * nA
        r = p.A() @ x - lam * (p.B() @ x)
        assert np.linalg.norm(r) / (nA * np.linalg.norm(x)) <= 1e-9
    P.close()
    c.close()
