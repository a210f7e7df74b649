"""GPU check of the Hellmann-Feynman backward at the largest workload size
(n = 1 492 992 tight-binding pencil, k = n/2): kth_eig, then the gradient of
lambda_k with respect to the stored values of A and B, checked by central
finite differences (h = 1e-6) of the forward on symmetric pairs of stored
entries, each difference forward warm-started from the first run's bracketing
interval and counts.  Entries: half drawn with probability proportional to
|x_i x_j| (the eigenvector is localised, so uniform picks mostly give
gradients near zero), half drawn uniformly; A and B alternate.  Also the inertia
bracket certificate of the returned eigenvalue and the homogeneity identities
sum_p gA[p] a_p = lambda, sum_p gB[p] b_p = -lambda.

KTH_FD_ENTRIES sets the number of entries (default 16; the workload's full
check uses 32).  Collected last: it is the longest GPU test (about four
minutes at 16 entries)."""
import os
import time

import numpy as np
import pytest

import pencilgen as pg
from tests.gpu_util import kth, note

pytestmark = pytest.mark.gpu


def _mirror(p, q, rows):
    """Index of the stored entry (j, i) for the stored entry q = (i, j)."""
    i, j = rows[q], p.col[q]
    lo, hi = p.rowptr[j], p.rowptr[j + 1]
    q2 = lo + int(np.searchsorted(p.col[lo:hi], i))
    assert p.col[q2] == i
    return q2


@pytest.mark.timeout(1200)
def test_hf_gradient_n1_5m_central_differences():
    K = kth()
    ctx = K.Context(0)
    p = pg.workload("n1_5m")
    n, k = p.n, p.k
    note(f"HF gradient n={n} k={k}: pencil")
    P = K.Pencil.from_pencilgen(ctx, p)
    sv = pg.start_vectors(n)
    t0 = time.perf_counter()
    lam, x, info = P.eig(k, start_vectors=sv)
    note(f"  kth_eig {time.perf_counter() - t0:.1f} s: lambda {lam!r}, validated {info['k_validated']}, "
         f"{info['n_factorizations']} factorizations, residual {info['rel_residual_normA']:.2e}")
    assert info["k_validated"] == k
    nA = float(np.add.reduceat(np.abs(p.a_val), p.rowptr[:-1]).max())
    A, B = p.A(), p.B()
    assert np.linalg.norm(A @ x - lam * (B @ x)) / (nA * np.linalg.norm(x)) <= 1e-9
    # bracket certificate: nu(lam - d) < k <= nu(lam + d) iff lambda_k lies in [lam - d, lam + d)
    d = 1e-10 * nA
    assert P.nu(lam - d) < k <= P.nu(lam + d)
    ga, gb = P.backward(lam, x, 1.0)
    assert abs(ga @ p.a_val - lam) <= 1e-10 * abs(lam)
    assert abs(gb @ p.b_val + lam) <= 1e-10 * abs(lam)

    rows = np.repeat(np.arange(n), np.diff(p.rowptr))
    upper = np.nonzero(rows < p.col)[0]
    w = np.abs(x[rows[upper]] * x[p.col[upper]])
    rng = np.random.default_rng(11)
    nfd = int(os.environ.get("KTH_FD_ENTRIES", "16"))
    weighted = rng.choice(upper, nfd - nfd // 2, replace=False, p=w / w.sum())
    uniform = rng.choice(upper, nfd // 2, replace=False)
    picks = list(weighted) + list(uniform)
    wi = [info["sigma_lower"], info["sigma_upper"]]
    wc = [info["nu_lower"], info["nu_upper"]]
    h = 1e-6
    worst = 0.0
    for e, q in enumerate(picks):
        q = int(q)
        q2 = _mirror(p, q, rows)
        on_b = e % 2 == 1
        vals = []
        for sgn in (1, -1):
            a, b = p.a_val, p.b_val
            if on_b:
                b = b.copy()
                b[q] += sgn * h
                b[q2] += sgn * h
            else:
                a = a.copy()
                a[q] += sgn * h
                a[q2] += sgn * h
            P.set_values(a, b)
            v, _, fi = P.eig(k, start_vectors=sv, want_x=False, warm_interval=wi, warm_counts=wc)
            assert fi["k_validated"] == k
            vals.append(v)
        fd = (vals[0] - vals[1]) / (2 * h)
        g = gb if on_b else ga
        an = g[q] + g[q2]
        err = abs(fd - an)
        worst = max(worst, err / (1e-7 + 1e-4 * abs(an)))
        note(f"  entry {e} ({'B' if on_b else 'A'} {rows[q]},{p.col[q]}; "
             f"{'weighted' if e < len(weighted) else 'uniform'}): fd {fd:.6e} hf {an:.6e} |diff| {err:.1e}")
        assert err <= 1e-7 + 1e-4 * abs(an), (e, rows[q], p.col[q], fd, an)
    P.set_values(p.a_val, p.b_val)
    note(f"  worst |fd - hf| / (1e-7 + 1e-4 |hf|) = {worst:.3f} over {len(picks)} entries")
