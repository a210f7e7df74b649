"""Write the stored expected values of the full-size parity tests.

Calls only the oracle (and the seeded input generator); nothing here touches
the GPU library.  Each job writes one JSON file next to this script:

  inertia_<config>_<sigma>.json   nu(sigma) of the workload by the plain-C sparse
                                  LDL^T (fixed shifts, chosen near the middle of
                                  the spectrum where k = n/2 lies)
  three_stage_<config>.json       lambda_k, interval, counts of the oracle's own
                                  three-stage run (Alg. 4)

Usage: python tests/golden/make_golden.py inertia n131k -3.0
       python tests/golden/make_golden.py three_stage n131k
"""
import json
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


def main(argv):
    job, cfg = argv[0], argv[1]
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
        t = time.perf_counter()
        r = o3.kth_eig(p)
        out = dict(config=cfg, n=p.n, k=p.k, lam=r.lam, sigma_lower=r.sigma_lower,
                   sigma_upper=r.sigma_upper, nu_lower=r.nu_lower, nu_upper=r.nu_upper,
                   sigmas=r.sigmas, nus=r.nus, rel_residual=r.rel_residual,
                   norm_a_inf=od.norm_inf(p), stage1_steps=r.stage1_steps,
                   bisection_steps=r.bisection_steps, si_steps=r.si_steps,
                   seconds=time.perf_counter() - t, source="oracle.three_stage.kth_eig")
        path = os.path.join(HERE, f"three_stage_{cfg}.json")
    else:
        raise SystemExit("unknown job " + job)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out.get("nu", out.get("lam")))


if __name__ == "__main__":
    main(sys.argv[1:])
