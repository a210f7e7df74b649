"""Write the stored expected values of the full-size parity tests.

Calls only the oracle (and the seeded input generator); nothing here touches
the GPU library.  Each job writes one JSON file next to this script:

  inertia_<config>_<sigma>.json   nu(sigma) of the workload by the plain-C sparse
                                  LDL^T (fixed shifts, chosen near the middle of
                                  the spectrum where k = n/2 lies)
  three_stage_<config>.json       lambda_k, interval, counts of the oracle's own
                                  three-stage run (Alg. 4)
  kth_oracle_<config>.json        lambda_k of a workload too large for a whole
                                  oracle three-stage run on one core: the oracle
                                  isolates it by multisection (Alg. 1' with several
                                  shifts per round, counts from parallel processes),
                                  runs its own shift-and-invert Lanczos (Alg. 3) on
                                  the isolating interval, and certifies the result
                                  by inertia (Section 2.1): nu(lam - eps) < k <=
                                  nu(lam + eps) proves lambda_k in [lam - eps,
                                  lam + eps).  Resumable: every finished round is
                                  written before the next starts.
  batch_dense_<count>.json        lambda_k of each pencil of uneven_batch(count) by
                                  the dense oracle (Cholesky reduction, eigenvalues)

Usage: python tests/golden/make_golden.py inertia n131k -3.0
       python tests/golden/make_golden.py three_stage n131k [bisection|interp]
       python tests/golden/make_golden.py kth_oracle n524k [workers]
       python tests/golden/make_golden.py batch_dense 256
"""
import glob
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import pencilgen as pg  # noqa: E402
from oracle import dense as od  # noqa: E402
from oracle import sparse as osp  # noqa: E402
from oracle import three_stage as o3  # noqa: E402


_SHARED = {}


def _init_worker(cfg):
    # each worker process builds the workload and the oracle's ordering itself
    _SHARED["P"] = osp.prepare(pg.workload(cfg))


def _count(sigma):
    st = osp.ldlt_stats(_SHARED["P"], sigma)
    return float(sigma), int(st.neg), int(st.zero)


def _counts(cfg, sigmas, workers):
    """Oracle inertia at several shifts, one process per shift (fresh processes:
    a forked child of a process that already ran threads can deadlock)."""
    with mp.get_context("spawn").Pool(min(workers, len(sigmas)), initializer=_init_worker,
                                       initargs=(cfg,)) as pool:
        return pool.map(_count, list(sigmas), chunksize=1)


def _save(path, state):
    with open(path + ".tmp", "w") as f:
        json.dump(state, f, indent=1)
    os.replace(path + ".tmp", path)


def kth_oracle(cfg, workers, m_max=20, first_step=0.0015):
    """Oracle-only lambda_k of a large workload (see the module docstring)."""
    p = pg.workload(cfg)
    P = osp.prepare(p)
    nA = od.norm_inf(p)
    k = p.k
    path = os.path.join(HERE, f"kth_oracle_{cfg}.json")
    if os.path.exists(path):
        state = json.load(open(path))
    else:
        state = dict(config=cfg, n=p.n, k=k, norm_a_inf=nA, m_max=m_max, counts=[],
                     phase="isolate", source="oracle.sparse.ldlt_stats + oracle.three_stage.stage3")
        # counts already computed by the oracle at fixed shifts
        for f in sorted(glob.glob(os.path.join(HERE, f"inertia_{cfg}_*.json"))):
            g = json.load(open(f))
            state["counts"].append([g["sigma"], g["nu"], g["zero"]])
    t_all = time.perf_counter()
    while state["phase"] != "done":
        good = [c for c in state["counts"] if c[2] == 0]
        below = [c for c in good if c[1] < k]
        above = [c for c in good if c[1] >= k]
        lo = max(below) if below else None
        hi = min(above) if above else None
        if state["phase"] == "isolate":
            if not good:
                # nothing known yet: probes spread over [-||A||, ||A||]
                pts = [nA * (2.0 * (i + 1) / (workers + 1) - 1.0) for i in range(workers)]
            elif lo is None or hi is None:
                # extend from the known side with growing steps
                step = first_step * (2 ** state.get("extend", 0))
                state["extend"] = state.get("extend", 0) + 1
                base = lo[0] if lo is not None else hi[0]
                sgn = 1.0 if lo is not None else -1.0
                pts = [base + sgn * step * (i + 1) for i in range(workers)]
            elif hi[1] - lo[1] <= m_max:
                state["phase"] = "si"
                state["interval"] = dict(sigma_lower=lo[0], sigma_upper=hi[0],
                                         nu_lower=lo[1], nu_upper=hi[1])
                _save(path, state)
                continue
            else:
                w = hi[0] - lo[0]
                pts = [lo[0] + w * (i + 1) / (workers + 1) for i in range(workers)]
        elif state["phase"] == "si":
            iv = state["interval"]
            t = time.perf_counter()
            A, B = p.A(), p.B()
            lam, x, j, sig, ib, ir, idf = o3.stage3(
                P, k, iv["sigma_lower"], iv["sigma_upper"], iv["nu_lower"], iv["nu_upper"],
                A, B, pg.start_vectors(p.n)[1])
            x = x / np.sqrt(np.dot(x, B @ x))
            r = A @ x - lam * (B @ x)
            state.update(lam=float(lam), sigma_si=float(sig), si_steps=int(j), it_bound=int(ib),
                         it_residual=int(ir), it_difference=int(idf),
                         rel_residual_normA=float(np.linalg.norm(r) / (nA * np.linalg.norm(x))),
                         si_seconds=time.perf_counter() - t, phase="certify")
            _save(path, state)
            continue
        else:   # certify
            lam = state["lam"]
            eps, dlt = 1e-11 * nA, 1e-10 * nA
            pts = [lam - dlt, lam - eps, lam + eps, lam + dlt]
        t = time.perf_counter()
        res = _counts(cfg, pts, workers)
        state["counts"].extend([list(r) for r in res])
        state.setdefault("rounds", []).append(dict(phase=state["phase"], sigmas=pts,
                                                   seconds=time.perf_counter() - t))
        if state["phase"] == "certify":
            lam = state["lam"]
            eps = 1e-11 * nA
            d = {r[0]: r for r in res}
            lo_c, hi_c = d[pts[1]], d[pts[2]]
            state["certificate"] = dict(
                eps=eps, sigma_minus=pts[1], nu_minus=lo_c[1], sigma_plus=pts[2],
                nu_plus=hi_c[1],
                holds=bool(lo_c[2] == 0 and hi_c[2] == 0 and lo_c[1] < k <= hi_c[1]))
            state["phase"] = "done"
        _save(path, state)
        print(state["phase"], len(state["counts"]), "counts", flush=True)
    state["counts"].sort()
    state["seconds_this_run"] = time.perf_counter() - t_all
    _save(path, state)
    return path, state.get("lam")


def batch_dense(count):
    out = dict(count=count, seed=0, source="oracle.dense.eigvals", pencils=[])
    t0 = time.perf_counter()
    for i, q in enumerate(pg.uneven_batch(count=count, seed=0)):
        lam = od.eigvals(q)
        out["pencils"].append(dict(i=i, n=q.n, k=q.k, lam=float(lam[q.k - 1]),
                                   gap_below=float(lam[q.k - 1] - lam[q.k - 2]),
                                   gap_above=float(lam[q.k] - lam[q.k - 1]),
                                   norm_a_inf=od.norm_inf(q)))
        print(i, q.n, flush=True)
    out["seconds"] = time.perf_counter() - t0
    path = os.path.join(HERE, f"batch_dense_{count}.json")
    _save(path, out)
    return path, len(out["pencils"])


def main(argv):
    job, cfg = argv[0], argv[1]
    if job == "kth_oracle":
        workers = int(argv[2]) if len(argv) > 2 else max(1, (os.cpu_count() or 2) - 1)
        print(*kth_oracle(cfg, workers))
        return
    if job == "batch_dense":
        print(*batch_dense(int(cfg)))
        return
    p = pg.workload(cfg)
    if job == "inertia":
        sigma = float(argv[2])
        t = time.perf_counter()
        st = osp.ldlt_stats(p, sigma)
        out = dict(config=cfg, n=p.n, sigma=sigma, nu=int(st.neg), zero=int(st.zero),
                   pos=int(st.pos), flops=st.flops, nnz_l=int(st.nnz_l),
                   seconds=time.perf_counter() - t, source="oracle.sparse.ldlt_stats")
        path = os.path.join(HERE, f"inertia_{cfg}_{sigma:+.3f}.json")
    elif job == "three_stage":
        rf = argv[2] if len(argv) > 2 else "bisection"
        t = time.perf_counter()
        r = o3.kth_eig(p, root_finder=rf)
        out = dict(config=cfg, n=p.n, k=p.k, lam=r.lam, sigma_lower=r.sigma_lower,
                   sigma_upper=r.sigma_upper, nu_lower=r.nu_lower, nu_upper=r.nu_upper,
                   sigmas=r.sigmas, nus=r.nus, rel_residual=r.rel_residual,
                   norm_a_inf=od.norm_inf(p), stage1_steps=r.stage1_steps,
                   bisection_steps=r.bisection_steps, si_steps=r.si_steps,
                   root_finder=rf, seconds=time.perf_counter() - t,
                   source="oracle.three_stage.kth_eig")
        path = os.path.join(HERE, f"three_stage_{cfg}.json" if rf == "bisection"
                            else f"three_stage_{cfg}_{rf}.json")
    else:
        raise SystemExit("unknown job " + job)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out.get("nu", out.get("lam")))


if __name__ == "__main__":
    main(sys.argv[1:])
