"""GPU checks of the rest of the C ABI: error paths, batched inertia and
pencils, device pointers, determinism, warm start, and the Hellmann-Feynman
backward against the oracle gradient and finite differences."""
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


def test_singular_shift(K, ctx):
    n = 12
    p = pg.Pencil(n=n, rowptr=np.arange(n + 1, dtype=np.int64), col=np.arange(n, dtype=np.int32),
                  a_val=np.arange(1.0, n + 1), b_val=np.ones(n))
    note("singular shift")
    P = K.Pencil.from_pencilgen(ctx, p)
    assert P.nu(4.5) == 4
    with pytest.raises(K.KthError) as e:
        P.inertia(4.0)
    assert e.value.status == K.KTH_ESINGULAR


def test_b_not_positive_definite(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=1)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    b = p.b_val.copy()
    b[(rows == p.col) & (rows == 5)] = -1.0
    note("B indefinite")
    P = K.Pencil(ctx, p.rowptr, p.col, p.a_val, b)
    with pytest.raises(K.KthError) as e:
        P.eig(p.n // 2)
    assert e.value.status == K.KTH_ENOTPD


def test_no_convergence_and_bad_k(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=2)
    note("ENOCONV / EINVAL")
    P = K.Pencil.from_pencilgen(ctx, p)
    with pytest.raises(K.KthError) as e:
        P.eig(p.n // 2, max_lanczos=3)
    assert e.value.status in (K.KTH_ENOCONV, K.KTH_ECLUSTER)
    for k in (0, p.n + 1):
        with pytest.raises(K.KthError) as e:
            P.eig(k)
        assert e.value.status == K.KTH_EINVAL


def test_inertia_batch_and_determinism(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    note("inertia batch")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, _ = od.eig(p)
    sig = np.linspace(lam[0] - 0.5, lam[-1] + 0.5, 33)
    nb = P.inertia_batch(sig)
    assert [P.nu(s) for s in sig] == nb.tolist() == [od.nu(lam, s) for s in sig]
    F1, F2 = P.factor(-3.0), P.factor(-3.0)
    b = np.random.default_rng(1).normal(size=p.n)
    assert np.array_equal(F1.solve(b), F2.solve(b))      # bit-identical repeats


def _hip():
    """The HIP runtime libkth.so itself links (same process-wide instance)."""
    import ctypes
    import glob
    path = sorted(glob.glob("/opt/rocm/lib/libamdhip64.so*"))[0]
    h = ctypes.CDLL(path)
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipDeviceSynchronize.argtypes = []
    return h


def test_solve_device_pointers(K, ctx):
    import ctypes
    p = pg.tb_supercell((3, 3, 3), seed=4)
    note("device-pointer solve")
    P = K.Pencil.from_pencilgen(ctx, p)
    F = P.factor(-2.0)
    b = np.asfortranarray(np.random.default_rng(2).normal(size=(p.n, 2)))
    xh = F.solve(b)
    hip = _hip()
    nbytes = b.nbytes
    bd, xd = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(bd), nbytes) == 0 and hip.hipMalloc(ctypes.byref(xd), nbytes) == 0
    try:
        assert hip.hipMemcpy(bd, b.ctypes.data, nbytes, 1) == 0          # host -> device
        K._check(K.lib().kth_solve(F.h, 2, bd.value, p.n, xd.value, p.n, K.KTH_DEVICE_PTRS), ctx.h)
        xo = np.zeros_like(b)
        assert hip.hipMemcpy(xo.ctypes.data, xd, nbytes, 2) == 0         # device -> host
        assert np.array_equal(xo, xh)
    finally:
        hip.hipFree(bd)
        hip.hipFree(xd)


def test_warm_start_and_batch(K, ctx):
    ps = [pg.tb_cluster(na, seed=np.random.SeedSequence(5).spawn(3)[i]) for i, na in enumerate((130, 211, 97))]
    note("eig batch")
    Ps = [K.Pencil.from_pencilgen(ctx, p) for p in ps]
    ks = [int(0.4 * p.n) for p in ps]
    res = K.eig_batch(ctx, Ps, ks)
    for p, k, (st, lam, x, info) in zip(ps, ks, res):
        assert st == K.KTH_OK
        lam_ref, _ = od.kth(p, k)
        assert info["k_validated"] == k
        assert abs(lam - lam_ref) <= 1e-10 * od.norm_inf(p)
    # warm start from the first run's interval gives the same eigenvalue
    st, lam0, _, info0 = res[0]
    lam1, _, info1 = Ps[0].eig(ks[0], warm_interval=[info0["sigma_lower"], info0["sigma_upper"]],
                               warm_counts=[info0["nu_lower"], info0["nu_upper"]])
    assert abs(lam1 - lam0) <= 1e-12 * od.norm_inf(ps[0])
    assert info1["bisection_steps"] == 0 and info1["stage1_steps"] == 0


def test_hellmann_feynman_backward(K, ctx):
    p = pg.tb_supercell((4, 4, 4), seed=0)
    k = p.n // 2
    note("HF backward")
    P = K.Pencil.from_pencilgen(ctx, p)
    lam, x, info = P.eig(k, start_vectors=pg.start_vectors(p.n))
    ga, gb = P.backward(lam, x, 1.0)
    lam_ref, x_ref = od.kth(p, k)
    ra, rb = od.hf_gradient(p, lam_ref, x_ref)
    scale = max(np.abs(ra).max(), np.abs(rb).max())
    assert np.abs(ga - ra).max() <= 1e-8 * scale
    assert np.abs(gb - rb).max() <= 1e-8 * scale
    # homogeneity: sum g_A a = lambda, sum g_B b = -lambda
    assert abs(ga @ p.a_val - lam) <= 1e-10 * abs(lam)
    assert abs(gb @ p.b_val + lam) <= 1e-10 * abs(lam)
    # central finite differences of the GPU forward on symmetric entry pairs
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    mag = np.abs(x[rows] * x[p.col])
    cand = np.nonzero((rows < p.col) & (mag > 1e-3 * mag.max()))[0]
    picks = np.random.default_rng(0).choice(cand, 4, replace=False)
    h = 1e-6
    sv = pg.start_vectors(p.n)
    for q in picks:
        i, j = rows[q], p.col[q]
        q2 = p.rowptr[j] + int(np.searchsorted(p.col[p.rowptr[j]:p.rowptr[j + 1]], i))
        vals = []
        for sgn in (1, -1):
            a = p.a_val.copy()
            a[q] += sgn * h
            a[q2] += sgn * h
            P.set_values(a, p.b_val)
            vals.append(P.eig(k, start_vectors=sv, want_x=False)[0])
        P.set_values(p.a_val, p.b_val)
        fd = (vals[0] - vals[1]) / (2 * h)
        an = ga[q] + ga[q2]
        assert abs(fd - an) <= 1e-7 + 1e-4 * abs(an), (i, j, fd, an)


def test_handle_release_order(K):
    # a kept factor stays usable after its pencil and context handles are destroyed
    p = pg.tb_supercell((2, 2, 2), seed=5)
    note("handle release order")
    c2 = K.Context(0)
    P = K.Pencil.from_pencilgen(c2, p)
    F = P.factor(-3.0)
    b = np.random.default_rng(2).normal(size=p.n)
    x_before = F.solve(b)
    c2.close()
    P.close()
    x_after = F.solve(b)
    assert np.array_equal(x_before, x_after)
    F.close()


def test_option_validation(K, ctx):
    p = pg.tb_supercell((2, 2, 2), seed=6)
    note("option validation")
    P = K.Pencil.from_pencilgen(ctx, p)
    for bad in (dict(multisection=0), dict(multisection=65), dict(m_max=-1), dict(ir_tol=-1.0),
                dict(si_precision=7), dict(max_lanczos=0), dict(tau_res=0.0), dict(root_finder=2),
                dict(root_finder=1, multisection=3), dict(si_block=65), dict(si_block=-1)):
        with pytest.raises(K.KthError) as e:
            P.eig(p.n // 2, **bad)
        assert e.value.status == K.KTH_EINVAL, bad


def _sub_pattern(p, keep):
    """CSR of the entries of p's pattern selected by the boolean mask keep."""
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    rp = np.zeros(p.n + 1, dtype=np.int64)
    np.add.at(rp, rows[keep] + 1, 1)
    return np.cumsum(rp), p.col[keep].astype(np.int32)


def test_separate_patterns(K, ctx):
    # B on its nonzero entries only, A on the full pattern (and the converse): the
    # union is the full pattern, so every result equals the shared-pattern pencil's
    p = pg.tb_supercell((2, 2, 3), seed=8)
    note("separate A / B patterns")
    full = K.Pencil.from_pencilgen(ctx, p)
    kb = p.b_val != 0.0
    ka = p.a_val != 0.0
    assert kb.sum() < p.nnz and ka.sum() < p.nnz
    brp, bcol = _sub_pattern(p, kb)
    arp, acol = _sub_pattern(p, ka)
    PB = K.Pencil(ctx, p.rowptr, p.col, p.a_val, p.b_val[kb], b_rowptr=brp, b_col=bcol)
    PA = K.Pencil(ctx, arp, acol, p.a_val[ka], p.b_val, b_rowptr=p.rowptr, b_col=p.col)
    lam, _ = od.eig(p)
    for s in np.linspace(lam[0] - 0.3, lam[-1] + 0.3, 9):
        assert full.nu(s) == PB.nu(s) == PA.nu(s) == od.nu(lam, s)
    k = p.n // 2
    sv = pg.start_vectors(p.n)
    l0, x0, _ = full.eig(k, start_vectors=sv)
    l1, x1, _ = PB.eig(k, start_vectors=sv)
    l2, x2, _ = PA.eig(k, start_vectors=sv)
    assert l0 == l1 == l2 and np.array_equal(x0, x1) and np.array_equal(x0, x2)
    ga0, gb0 = full.backward(l0, x0)
    ga1, gb1 = PB.backward(l0, x0)
    ga2, gb2 = PA.backward(l0, x0)
    assert np.array_equal(ga1, ga0) and np.array_equal(gb1, gb0[kb])
    assert np.array_equal(ga2, ga0[ka]) and np.array_equal(gb2, gb0)
    # new values on the separate patterns: the spectrum doubles
    PB.set_values(2.0 * p.a_val, p.b_val[kb])
    for s in np.linspace(2 * lam[0] - 0.3, 2 * lam[-1] + 0.3, 7):
        assert PB.nu(s) == od.nu(2.0 * lam, s)


def test_pencil_create_device_pointers(K, ctx):
    import ctypes
    p = pg.tb_supercell((2, 2, 2), seed=9)
    note("device-pointer pencil create")
    host = K.Pencil.from_pencilgen(ctx, p)
    hip = _hip()
    arrs = [np.ascontiguousarray(p.rowptr, dtype=np.int64), np.ascontiguousarray(p.col, dtype=np.int32),
            np.ascontiguousarray(p.a_val), np.ascontiguousarray(p.b_val)]
    dev = [ctypes.c_void_p() for _ in arrs]
    try:
        for a, d in zip(arrs, dev):
            assert hip.hipMalloc(ctypes.byref(d), a.nbytes) == 0
            assert hip.hipMemcpy(d, a.ctypes.data, a.nbytes, 1) == 0
        h = ctypes.c_void_p()
        P64, P32, PD = (ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_double))
        K._check(K.lib().kth_pencil_create(
            ctx.h, p.n, ctypes.cast(dev[0].value, P64), ctypes.cast(dev[1].value, P32),
            ctypes.cast(dev[2].value, PD), ctypes.cast(dev[0].value, P64), ctypes.cast(dev[1].value, P32),
            ctypes.cast(dev[3].value, PD), K.KTH_DEVICE_PTRS, ctypes.byref(h)), ctx.h)
        try:
            for s in (-4.0, -2.5, 0.5):
                nu, nz = ctypes.c_int64(), ctypes.c_int64()
                K._check(K.lib().kth_inertia(h, s, ctypes.byref(nu), ctypes.byref(nz)), ctx.h)
                assert nu.value == host.nu(s)
        finally:
            K.lib().kth_pencil_destroy(h)
    finally:
        for d in dev:
            hip.hipFree(d)
