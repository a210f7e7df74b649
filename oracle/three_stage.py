"""Oracle (test infrastructure only): the three-stage algorithm (Alg. 4) in FP64.

Alg. 2 (initial interval from extreme Ritz values), Alg. 1' (bisection with a
sparse LDL^T inertia count) and Alg. 3 (shift-and-invert Lanczos with error
bounds, Prop. 3), written from the paper's description over the plain-C
sparse oracle for nu(sigma) and the linear solves, and scipy's CSR product for
A x and B x.  Readings of points the paper leaves open:

* starting vectors come from ``pencilgen.start_vectors`` (row 0: stage 1,
  row 1: stage 3, later rows: restarts after a breakdown);
* both Lanczos processes use full two-pass classical Gram-Schmidt
  reorthogonalisation in their inner product;
* the SI basis is kept as V = B^{-1} V~ (B-orthonormal) together with V~ = B V,
  so B^{-1} is never applied; x_{i,2} = theta_i V y_i + beta_j (e_j^T y_i) v_{j+1},
  which equals (A - sigma B)^{-1} V~ y_i by the SI Lanczos decomposition;
* the m pairs nearest sigma are those with the largest |theta~| (ties: larger
  theta~ first); inclusion uses the closed bound inside [sigma_l, sigma_u);
* relative differences pair the m validated vectors of consecutive iterations in
  ascending eigenvalue order, after scaling to unit 2-norm and aligning signs;
* the residual test uses eq. (res2): ||r_{i,2}|| = |s_i| ||v~_{j+1}||;
* the returned vector is B-normalised with its largest-|.| entry positive.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import pencilgen
from . import sparse as osp


@dataclasses.dataclass
class Result:
    lam: float
    x: np.ndarray
    k_validated: int
    sigma_lower: float
    sigma_upper: float
    nu_lower: int
    nu_upper: int
    sigma_si: float
    stage1_steps: int
    bisection_steps: int
    si_steps: int
    it_bound: int
    it_residual: int
    it_difference: int
    sigmas: list          # every shift whose inertia was computed, in order
    nus: list
    rel_residual: float   # ||(A - lam B) x||_2 / ||x||_2 with explicit products
    n_factorizations: int
    si_block: int = 1     # block size of the shift-and-invert Lanczos that validated


class NoConvergence(RuntimeError):
    pass


def _bnorm(Bx, x):
    return float(np.sqrt(np.dot(x, Bx)))


def _tridiag_eig(alpha, beta):
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    return np.linalg.eigh(T)


def stage1(pencil, k, P, A, B, Bfac, v0s, nu_of, log):
    """Alg. 2: returns sigma_l, sigma_u, nu_l, nu_u, steps."""
    restart = 0
    v = v0s[0].copy()
    Bv = B @ v
    nb = _bnorm(Bv, v)
    V, BV = [v / nb], [Bv / nb]
    alphas, betas = [], []
    sig_prev, nu_prev = None, 0
    j = 0
    while True:
        j += 1
        vj, Bvj = V[-1], BV[-1]
        Av = A @ vj
        alphas.append(float(np.dot(vj, Av)))
        w = Bfac.solve(Av)       # B^{-1} A v_j
        Bw = Av.copy()
        Vm, BVm = np.array(V).T, np.array(BV).T
        for _ in range(2):       # CGS2 in the B inner product
            h = Vm.T @ Bw
            w -= Vm @ h
            Bw -= BVm @ h
        theta = np.linalg.eigvalsh(np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1))
        sig = float(theta[0]) if k <= nu_prev else float(theta[-1])
        nu = nu_of(sig)
        log.append((sig, nu))
        if j != 1 and (nu < k <= nu_prev or nu_prev < k <= nu):
            return min(sig_prev, sig), max(sig_prev, sig), min(nu_prev, nu), max(nu_prev, nu), j
        sig_prev, nu_prev = sig, nu
        beta = _bnorm(Bw, w)
        if beta <= 1e-14 * max(1.0, abs(alphas[-1])):
            # breakdown: restart with the next seeded vector
            restart += 1
            if restart >= v0s.shape[0] - 1:
                raise NoConvergence("stage-1 Lanczos broke down repeatedly")
            v = v0s[1 + restart].copy()
            Bv = B @ v
            nb = _bnorm(Bv, v)
            V, BV = [v / nb], [Bv / nb]
            alphas, betas = [], []
            sig_prev, nu_prev, j = None, 0, 0
            continue
        betas.append(beta)
        V.append(w / beta)
        BV.append(Bw / beta)
        if j > P.n + 1:
            raise NoConvergence("stage-1 exceeded n steps")


def stage2(k, sl, su, nl, nu_, nu_of, log, m_max=20, tau_len=0.0):
    """Alg. 1': bisection until nu_u - nu_l <= m_max (repeat-until, i.e. at least
    one step), or the interval is shorter than tau_len (cluster guard)."""
    steps = 0
    while True:
        sig = 0.5 * (sl + su)
        nu = nu_of(sig)
        log.append((sig, nu))
        steps += 1
        if k <= nu:
            su, nu_ = sig, nu
        else:
            sl, nl = sig, nu
        if nu_ - nl <= m_max:
            break
        if tau_len > 0 and (su - sl) < tau_len:
            break
    return sl, su, nl, nu_, steps


def interp_shift(k, sl, su, nl, nu_, m_max):
    """The next shift of the interpolating stage 2 (a bracketing root-finder on
    the counting function, Section 2.1 and Section 5 name such methods as
    alternatives to bisection).  nu(sigma) is modelled as linear between the
    bracket ends; the shift aims at the count that would bring the farther end
    to within m_max / 2 of k: k - m_max/2 for the lower end, k + m_max/2 - 1 for
    the upper one, plus 1/2 to land inside the count's step.  The fraction of
    the bracket is kept inside [1/64, 63/64]."""
    if (k - nl) >= (nu_ - k):
        c = k - m_max / 2.0 + 0.5
    else:
        c = k + m_max / 2.0 - 1.0 + 0.5
    t = (c - nl) / (nu_ - nl)
    t = min(max(t, 1.0 / 64.0), 63.0 / 64.0)
    return sl + t * (su - sl)


def stage2_interp(k, sl, su, nl, nu_, nu_of, log, m_max=20, tau_len=0.0):
    """Stage 2 with a safeguarded interpolating root-finder instead of the
    midpoint: the shift comes from interp_shift, except that after two
    consecutive interpolated steps that each failed to halve the count in the
    bracket (nu_u - nu_l) the next shift is the midpoint (a bisection step), which
    bounds the worst case.  Same stopping rule as Alg. 1' (at least one step;
    stop at nu_u - nu_l <= m_max, or below tau_len)."""
    steps = 0
    slow = []           # per interpolated step since the last bisection: gap not halved
    while True:
        bisect = len(slow) >= 2 and slow[-1] and slow[-2]
        sig = 0.5 * (sl + su) if bisect else interp_shift(k, sl, su, nl, nu_, m_max)
        gap = nu_ - nl
        nu = nu_of(sig)
        log.append((sig, nu))
        steps += 1
        if k <= nu:
            su, nu_ = sig, nu
        else:
            sl, nl = sig, nu
        slow = [] if bisect else slow + [2 * (nu_ - nl) > gap]
        if nu_ - nl <= m_max:
            break
        if tau_len > 0 and (su - sl) < tau_len:
            break
    return sl, su, nl, nu_, steps


def alg1_bisection(k, sl, su, nu_of, tau=None, rel_tau=None):
    """Alg. 1: plain spectral bisection until the interval is shorter than tau
    (absolute), or, as in the straightforward variant of Section 4.3.2, until
    (sigma_u - sigma_l) / max(|sigma_l|, |sigma_u|) < rel_tau.  Returns the
    midpoint estimate, the final interval and the number of steps."""
    steps = 0
    while True:
        w = su - sl
        if tau is not None and w < tau:
            break
        if rel_tau is not None and w / max(abs(sl), abs(su)) < rel_tau:
            break
        sig = 0.5 * (sl + su)
        if k <= nu_of(sig):
            su = sig
        else:
            sl = sig
        steps += 1
    return 0.5 * (sl + su), sl, su, steps


def stage3(pencil, k, sl, su, nl, nu_, A, B, v0, tau_res=1e-10, tau_diff=1e-10,
           max_iter=500, factor=None, trace=None):
    """Alg. 3: shift-and-invert Lanczos at the midpoint with validated index.
    ``trace`` (optional) is called at every iteration j >= m with the Ritz data."""
    l = k - nl
    m = nu_ - nl
    sigma = 0.5 * (sl + su)
    F = factor if factor is not None else osp.Factor(pencil, sigma)
    v = v0.copy()
    Bv = B @ v
    nb = _bnorm(Bv, v)
    V, Vt = [v / nb], [Bv / nb]             # V = B^{-1} V~, V~ = B V
    alphas, betas = [], []
    prev = None
    it_bound = it_res = it_diff = 0
    for j in range(1, max_iter + 1):
        w = F.solve(Vt[-1])                  # (A - sigma B)^{-1} v~_j
        Bw = B @ w
        Vm, Vtm = np.array(V).T, np.array(Vt).T
        h = Vtm.T @ w                        # = V^T B w
        alphas.append(float(h[-1]))
        w -= Vm @ h
        Bw -= Vtm @ h
        h2 = Vtm.T @ w
        w -= Vm @ h2
        Bw -= Vtm @ h2
        beta = float(np.sqrt(max(np.dot(w, Bw), 0.0)))
        if beta > 0:
            vnext, vtnext = w / beta, Bw / beta
        else:
            vnext, vtnext = np.zeros_like(w), np.zeros_like(w)
        if j >= m:
            th, Y = _tridiag_eig(np.array(alphas), np.array(betas))
            order = sorted(range(j), key=lambda i: (-abs(th[i]), -th[i]))[:m]
            lam = sigma + 1.0 / th[order]
            s = beta * Y[-1, order] / th[order]
            eta = (1.0 / np.abs(th[order])) * np.abs(s) / np.sqrt(1.0 + s * s)
            X = Vm @ (Y[:, order] * th[order]) + np.outer(vnext, beta * Y[-1, order])
            incl = bool(np.all(lam - eta >= sl) and np.all(lam + eta < su))
            asc = np.argsort(lam, kind="stable")
            lo, hi = (lam - eta)[asc], (lam + eta)[asc]
            disj = bool(np.all(hi[:-1] < lo[1:]))
            xn = np.linalg.norm(X, axis=0)
            rres = np.abs(s) * np.linalg.norm(vtnext) / xn
            res_ok = bool(np.all(rres < tau_res))
            Xa = X[:, asc] / xn[asc]
            if prev is not None:
                sg = np.sign(np.sum(Xa * prev, axis=0))
                sg[sg == 0] = 1.0
                diff = np.linalg.norm(Xa * sg - prev, axis=0)
                diff_ok = bool(np.all(diff < tau_diff))
            else:
                diff_ok = False
            prev = Xa
            if trace is not None:
                trace(dict(j=j, sigma=sigma, theta=th, Y=Y, order=order, lam=lam, eta=eta,
                           s=s, X=X, V=Vm, Vt=Vtm, vnext=vnext, vtnext=vtnext, beta=beta,
                           incl=incl, disj=disj, res_ok=res_ok, diff_ok=diff_ok))
            if incl and disj and not it_bound:
                it_bound = j
            if res_ok and not it_res:
                it_res = j
            if diff_ok and not it_diff:
                it_diff = j
            if incl and disj and res_ok and diff_ok:
                lam_asc = lam[asc]
                x = X[:, asc[l - 1]].copy()
                return (float(lam_asc[l - 1]), x, j, sigma, it_bound, it_res, it_diff)
        if beta == 0:
            raise NoConvergence("SI Lanczos reached an invariant subspace before validation")
        betas.append(beta)
        V.append(vnext)
        Vt.append(vtnext)
    raise NoConvergence("SI Lanczos did not converge")


def _b_orthonormalize(X, BX):
    """X R^{-1}, BX R^{-1} with X^T B X = R^T R (Cholesky), twice (CholQR2), and
    the total factor R (upper triangular)."""
    Rt = np.eye(X.shape[1])
    for _ in range(2):
        G = X.T @ BX
        G = 0.5 * (G + G.T)
        try:
            R = np.linalg.cholesky(G).T
        except np.linalg.LinAlgError:
            raise NoConvergence("block Lanczos: the new block is rank deficient")
        X = np.linalg.solve(R.T, X.T).T
        BX = np.linalg.solve(R.T, BX.T).T
        Rt = R @ Rt
    return X, BX, Rt


def _components(lam, eta, asc):
    """Groups of consecutive (ascending) Ritz values whose closed bounds
    [lam - eta, lam + eta] overlap."""
    comps, cur = [], [asc[0]]
    for a, b in zip(asc[:-1], asc[1:]):
        if lam[a] + eta[a] >= lam[b] - eta[b]:
            cur.append(b)
        else:
            comps.append(cur)
            cur = [b]
    comps.append(cur)
    return comps


def stage3_block(pencil, k, sl, su, nl, nu_, A, B, V0, tau_res=1e-10, tau_diff=1e-10,
                 max_iter=500, factor=None, scale=None):
    """Block shift-and-invert Lanczos for an interval that may hold multiple or
    clustered eigenvalues (Section 3.4 names this modification; block size p =
    V0.shape[1]).  With V = B^{-1} V~ kept B-orthonormal and V~ = B V:
        (A - sigma B)^{-1} B V_j = V_j T_j + V_{j+1} B_j E_j^T,
    T_j block tridiagonal (diagonal blocks A_i, subdiagonal blocks B_i upper
    triangular from the B-orthonormalisation of each new block).  For a Ritz pair
    (theta, y) of T_j: lambda = sigma + 1/theta, x_2 = theta V_j y + V_{j+1} B_j
    E_j^T y = (A - sigma B)^{-1} V~_j y, residual (A - lambda B) x_2 = -V~_{j+1} s with
    s = B_j E_j^T y / theta, so Prop. 3 holds with |s| replaced by ||s||_2.
    Validation (Alg. 3 modified for multiplicity): the m pairs of largest |theta|;
    every bound inside [sigma_l, sigma_u); bounds that overlap form a cluster C,
    for which the B-orthonormal Ritz vectors V_j Y_C of the operator
    (A - sigma B)^{-1} B (self-adjoint in the B inner product) have residual norm
    rho = ||B_j E_j^T Y_C||_2, so (Kahan's theorem) |C| eigenvalues of the operator
    lie within rho of the theta's, i.e. within rho / (|theta| (|theta| - rho)) of
    the lambda's; cluster intervals and single bounds must be pairwise disjoint,
    which accounts for all m eigenvalues of the interval.  Residual test per pair;
    difference test per single pair as in Alg. 3, per cluster on its eigenvalues
    (|lambda^(j) - lambda^(j-1)| <= tau_diff max(1, |lambda|), same cluster shape).
    The bounds hold for the operator as applied; the factor's solves carry a
    backward error of order eps ||A - sigma B||, so bounds and cluster radii are
    not taken below 64 eps scale (scale = ||A||_inf + |sigma| ||B||_inf): the two
    computed copies of a multiple eigenvalue then stay one cluster."""
    l = k - nl
    m = nu_ - nl
    sigma = 0.5 * (sl + su)
    F = factor if factor is not None else osp.Factor(pencil, sigma)
    p = V0.shape[1]
    if scale is None:
        scale = (np.abs(A).sum(axis=1).max() + abs(sigma) * np.abs(B).sum(axis=1).max())
    floor = 64.0 * np.finfo(float).eps * float(scale)
    X, BX, _ = _b_orthonormalize(V0.copy(), B @ V0)
    V, Vt, Ad, Bd = [X], [BX], [], []
    prev = None
    it_bound = it_res = it_diff = 0
    for j in range(1, max_iter + 1):
        W = np.column_stack([F.solve(Vt[-1][:, c]) for c in range(p)])
        BW = B @ W
        Vm, Vtm = np.hstack(V), np.hstack(Vt)
        H = Vtm.T @ W
        Ad.append(0.5 * (H[-p:] + H[-p:].T))
        W -= Vm @ H
        BW -= Vtm @ H
        H2 = Vtm.T @ W
        W -= Vm @ H2
        BW -= Vtm @ H2
        Wn, BWn, Rn = _b_orthonormalize(W, BW)
        if j * p >= m:
            T = np.zeros((j * p, j * p))
            for i in range(j):
                T[i * p:(i + 1) * p, i * p:(i + 1) * p] = Ad[i]
                if i + 1 < j:
                    T[(i + 1) * p:(i + 2) * p, i * p:(i + 1) * p] = Bd[i]
                    T[i * p:(i + 1) * p, (i + 1) * p:(i + 2) * p] = Bd[i].T
            th, Y = np.linalg.eigh(T)
            sel = np.array(sorted(range(j * p), key=lambda i: (-abs(th[i]), -th[i]))[:m])
            ts = th[sel]
            lam = sigma + 1.0 / ts
            Yl = Y[-p:, sel]
            S = (Rn @ Yl) / ts
            sn = np.linalg.norm(S, axis=0)
            eta = np.maximum((1.0 / np.abs(ts)) * sn / np.sqrt(1.0 + sn * sn), floor)
            X = Vm @ (Y[:, sel] * ts) + Wn @ (Rn @ Yl)
            incl = bool(np.all(lam - eta >= sl) and np.all(lam + eta < su))
            asc = np.argsort(lam, kind="stable")
            comps = _components(lam, eta, asc)
            ivals, ok = [], incl
            for C in comps:
                if len(C) == 1:
                    q = C[0]
                    ivals.append((lam[q] - eta[q], lam[q] + eta[q]))
                    continue
                rho = float(np.linalg.norm(Rn @ Yl[:, C], 2))
                tc = np.abs(ts[C])
                if rho >= tc.min():
                    ok = False
                    break
                eps = np.maximum(rho / (tc * (tc - rho)), floor)
                ivals.append((float(np.min(lam[C] - eps)), float(np.max(lam[C] + eps))))
            if ok:
                ok = all(lo >= sl and hi < su for lo, hi in ivals) and \
                    all(ivals[i][1] < ivals[i + 1][0] for i in range(len(ivals) - 1))
            xn = np.linalg.norm(X, axis=0)
            rres = np.linalg.norm(BWn @ S, axis=0) / xn
            res_ok = bool(np.all(rres < tau_res))
            shape = tuple(len(C) for C in comps)
            Xa = X[:, asc] / xn[asc]
            la = lam[asc]
            diff_ok = False
            if prev is not None and prev[2] == shape:
                pX, pl, _ = prev
                diff_ok, pos = True, 0
                for c in shape:
                    if c == 1:
                        sg = 1.0 if np.dot(Xa[:, pos], pX[:, pos]) >= 0 else -1.0
                        diff_ok &= bool(np.linalg.norm(sg * Xa[:, pos] - pX[:, pos]) < tau_diff)
                    else:
                        seg = slice(pos, pos + c)
                        diff_ok &= bool(np.all(np.abs(la[seg] - pl[seg])
                                               <= tau_diff * np.maximum(1.0, np.abs(la[seg]))))
                    pos += c
            prev = (Xa, la, shape)
            if ok and not it_bound:
                it_bound = j
            if res_ok and not it_res:
                it_res = j
            if diff_ok and not it_diff:
                it_diff = j
            if ok and res_ok and diff_ok:
                return (float(la[l - 1]), X[:, asc[l - 1]].copy(), j, sigma, it_bound, it_res,
                        it_diff)
        V.append(Wn)
        Vt.append(BWn)
        Bd.append(Rn)
    raise NoConvergence("block SI Lanczos did not converge")


def block_start(n, p, seed=0):
    """Start block of the block shift-and-invert Lanczos: column 0 is row 1 of
    pencilgen.start_vectors (the single-vector start), columns 1.. rows 4.."""
    sv = pencilgen.start_vectors(n, seed=seed, count=max(4, p + 3))
    return np.column_stack([sv[1]] + [sv[3 + c] for c in range(1, p)])


def kth_eig(pencil, k: int | None = None, m_max=20, tau_res=1e-10, tau_diff=1e-10,
            tau_len=0.0, seed=0, max_iter=500, root_finder="bisection", si_block=0) -> Result:
    """Alg. 4 over the oracle's sparse LDL^T.  root_finder: "bisection" (Alg. 1')
    or "interp" (stage2_interp) for stage 2.  si_block: 1 the single-vector
    Alg. 3; p > 1 the block method (stage3_block) with block size p; 0 (default)
    Alg. 3 within 3 m + 30 steps, then the block method with p = m (a multiple
    eigenvalue leaves Alg. 3 one Ritz value short, Section 3.4), and the block
    method at once if stage 2 stopped on tau_len with more than m_max eigenvalues."""
    k = pencil.k if k is None else k
    P = osp.prepare(pencil)
    A, B = pencil.A(), pencil.B()
    v0s = pencilgen.start_vectors(pencil.n, seed=seed)
    # factor of B itself: the pencil (B, 0) at sigma = 0
    PB = osp.prepare(pencilgen.Pencil(n=pencil.n, rowptr=pencil.rowptr, col=pencil.col,
                                      a_val=pencil.b_val, b_val=np.zeros_like(pencil.b_val)),
                     perm=P.perm)
    Bfac = osp.Factor(PB, 0.0)
    if Bfac.inertia[0] or Bfac.inertia[1]:
        raise ValueError("B is not positive definite")
    nfac = [1]
    log = []

    def nu_of(s):
        nfac[0] += 1
        return osp.nu(P, s)

    sl, su, nl, nu_, s1 = stage1(pencil, k, P, A, B, Bfac, v0s, nu_of, log)
    if root_finder == "interp":
        sl, su, nl, nu_, s2 = stage2_interp(k, sl, su, nl, nu_, nu_of, log, m_max, tau_len)
    elif root_finder == "bisection":
        sl, su, nl, nu_, s2 = stage2(k, sl, su, nl, nu_, nu_of, log, m_max, tau_len)
    else:
        raise ValueError(f"unknown root finder {root_finder!r}")
    nfac[0] += 1
    m = nu_ - nl
    F = osp.Factor(P, 0.5 * (sl + su))
    block = si_block if si_block > 1 else 0
    if si_block == 0 and m > m_max:
        block = m
    res = None
    if block == 0:
        try:
            res = stage3(P, k, sl, su, nl, nu_, A, B, v0s[1], tau_res, tau_diff,
                         max_iter if si_block == 1 else min(max_iter, 3 * m + 30), factor=F)
        except NoConvergence:
            if si_block == 1:
                raise
            block = m
    if res is None:
        res = stage3_block(P, k, sl, su, nl, nu_, A, B, block_start(pencil.n, block, seed),
                           tau_res, tau_diff, max_iter, factor=F)
    lam, x, sj, sig, ib, ir, idf = res
    x = x / np.sqrt(np.dot(x, B @ x))
    i = int(np.argmax(np.abs(x)))
    if x[i] < 0:
        x = -x
    r = A @ x - lam * (B @ x)
    return Result(lam=lam, x=x, k_validated=k, sigma_lower=sl, sigma_upper=su, nu_lower=nl,
                  nu_upper=nu_, sigma_si=sig, stage1_steps=s1, bisection_steps=s2, si_steps=sj,
                  it_bound=ib, it_residual=ir, it_difference=idf,
                  sigmas=[a for a, _ in log], nus=[b for _, b in log],
                  rel_residual=float(np.linalg.norm(r) / np.linalg.norm(x)),
                  n_factorizations=nfac[0], si_block=max(block, 1))
