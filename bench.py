#!/usr/bin/env python3
"""Time-to-validated lambda_k on one MI355X, and the LDL^T rate.

Workload: the n = 524288 diamond tight-binding pencil (32 x 32 x 16 conventional
cells, 4 orbitals per atom, seed 0), k = n/2.  One step = one call of the
three-stage algorithm (Alg. 4) through the C ABI: B factor, stage-1 Lanczos with
its inertia counts, stage-2 bisection, the shift-and-invert factor and Lanczos
with validated index.  The pencil (pattern analysis, values) is resident on the
device before the timed region; the cold analysis time is reported apart.

Printed: one JSON line with the step time (`value`, seconds, lower is better),
the LDL^T GFLOP/s of one factorization at the first bisection shift, the
roofline of the dominant kernel (k_gemm_lt, the FP64-MFMA left-looking and
contribution-block products) from HIP events around its launches, and the CPU
oracle timed on a bounded sample of the same workload.  Extra legs (each
skippable with --skip): `hbm` (event-timed solve and SpMV bandwidth at the
shift-and-invert shift), `fp32_ir` (the same run with the FP32 shift-and-invert
factor and FP64 refinement), `c3a` (64 shifts of the n = 131072 pencil per
round against one at a time and against bisection), `c3b` (256 uneven pencils
in one batched call against a loop of single calls).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-validated λ_k (s) at n=524288; LDLᵀ GFLOP/s vs FP64-MFMA peak"
PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


# front-size classes (rows of the front) for the CPU baseline's sample
CPU_CLASSES = (0, 128, 512, 2048, 8192, 1 << 40)


def _front_flops(nf, ns):
    """sum over the ns pivot columns of c^2 + 2c, c = nf - 1 - j (vectorised)."""
    import numpy as np
    hi = nf.astype(np.float64) - 1.0          # c of the first pivot
    lo = hi - ns.astype(np.float64) + 1.0     # c of the last
    s1 = lambda m: m * (m + 1.0) / 2.0
    s2 = lambda m: m * (m + 1.0) * (2.0 * m + 1.0) / 6.0
    return (s2(hi) - s2(lo - 1.0)) + 2.0 * (s1(hi) - s1(lo - 1.0))


def cpu_baseline(pencil, n_factorizations: int, per_class=4, sample_flops=1.5e9):
    """The oracle's sparse LDL^T, projected from a bounded sample: its own ordering
    and symbolic analysis are timed whole; its partial factorization of a front
    (the flop sink) is timed on synthetic fronts of the workload's own shapes, a
    few per front-size class (the largest fronts capped at `sample_flops` of their
    first pivots), and each class's rate weights that class's share of the flops."""
    import numpy as np
    from oracle import sparse as osp
    t0 = time.perf_counter()
    P = osp.prepare(pencil)
    t_order = time.perf_counter() - t0
    t0 = time.perf_counter()
    shapes, F = osp.front_shapes(P)
    t_sym = time.perf_counter() - t0
    nf, ns = shapes[:, 0], shapes[:, 1]
    fl = _front_flops(nf, ns)
    per_fact = t_sym
    parts, t_sample = [], 0.0
    for lo, hi in zip(CPU_CLASSES[:-1], CPU_CLASSES[1:]):
        idx = np.nonzero((nf >= lo) & (nf < hi))[0]
        if idx.size == 0:
            continue
        fc = float(fl[idx].sum())
        order = idx[np.argsort(fl[idx], kind="stable")]
        picks = order[np.unique(np.linspace(0, order.size - 1, per_class).round().astype(int))]
        secs = flops = 0.0
        for q in picks:
            a, b = int(nf[q]), int(ns[q])
            # pivot cap: the first pivots of the front within sample_flops
            c = np.arange(a - 1, a - 1 - b, -1, dtype=np.float64)
            cum = np.cumsum(c * c + 2 * c)
            cap = int(np.searchsorted(cum, sample_flops)) + 1
            cap = 0 if cap >= b else cap
            s_, f_ = osp.front_sample(a, b, cap)
            secs += s_
            flops += f_
        rate = flops / max(secs, 1e-12)
        t_sample += secs
        per_fact += fc / rate
        parts.append(f"nf [{lo},{min(hi, int(nf.max()) + 1)}): {idx.size} fronts, "
                     f"{fc / F:.3f} of flops, {rate / 1e9:.2f} GFLOP/s")
    projected = t_order + n_factorizations * per_fact
    model, ncpu = _cpu_info()
    return {
        "value": projected, "unit": "s (projected)", "cores": 1, "kind": "oracle",
        "host": f"{model}, {ncpu} logical CPUs",
        "per_factorization_s": per_fact,
        "sample": (f"oracle ordering {t_order:.1f} s and symbolic {t_sym:.1f} s of the n={pencil.n} "
                   f"pencil timed whole; its front partial factorization timed on synthetic "
                   f"fronts of the workload's shapes, {per_class} per size class "
                   f"({t_sample:.1f} s of samples, largest fronts capped at {sample_flops:.1e} flops "
                   f"of their first pivots): " + "; ".join(parts) +
                   f"; projected x{n_factorizations} factorizations (assembly, extend-add, "
                   f"solves and Lanczos not counted)"),
    }


KERNEL_SOURCES = ("paper_1710_05134_amd/csrc/factor.hip", "paper_1710_05134_amd/csrc/device.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_lt_n524k_traffic.md")
PMC_SIGMA = -3.0
COPY_DOUBLES = 2 ** 27          # calibration copy: 1 GiB read + 1 GiB written


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def gemm_traffic():
    """HBM bytes per k_gemm_lt launch from the committed counter summary, or None if
    it is missing or was taken on other kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip("` ")] = v.strip().strip("`")
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(kv["k_gemm_lt_hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def pmc_sample():
    """One FP64 factorization of the bench pencil at sigma = PMC_SIGMA, a kept factor
    with three solves and three SpMV of each kind, then a plain 1 GiB device copy
    that calibrates FETCH_SIZE / WRITE_SIZE (run under rocprofv3 --pmc)."""
    import torch
    import pencilgen as pg
    import paper_1710_05134_amd as K
    torch.cuda.init()
    p = pg.workload("n524k")
    ctx = K.Context(0)
    P = K.Pencil.from_pencilgen(ctx, p)
    nu = P.nu(PMC_SIGMA)
    log(f"factorization at sigma={PMC_SIGMA}: nu={nu}")
    # a kept factor, three solves, three products B x and three fused A x, B x
    F = P.factor(PMC_SIGMA)
    pr = F.profile_solve(3)
    F.close()
    log(f"solve {pr['solve_s'] * 1e3:.2f} ms, B x {pr['spmv_b_s'] * 1e6:.1f} us")
    x = torch.empty(COPY_DOUBLES, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_sample": "n524k", "sigma": PMC_SIGMA, "nu": nu,
                      "copy_bytes": 8 * COPY_DOUBLES}), flush=True)


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize(stats_csv, fetch_csv, write_csv, command, pmc_command):
    """Markdown summary of a rocprofv3 kernel-stats CSV and, if given, of the
    FETCH_SIZE / WRITE_SIZE counter CSVs of a --pmc-sample run."""
    out = []
    if stats_csv:
        rows = _read_csv(stats_csv)
        out += ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
                "| kernel | calls | avg µs | total ms | % |", "|---|---|---|---|---|"]
        for r in rows[:15]:
            name = r["Name"].replace("kth::(anonymous namespace)::", "")
            name = name.split("(")[0] if "kth" in r["Name"] else name[:60]
            out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f} |")
        out.append("")
    if fetch_csv and write_csv:
        def per_kernel(path):
            acc = {}   # name -> [sum of bytes, dispatches, largest single dispatch]
            for r in _read_csv(path):
                nm = r["Kernel_Name"]
                v = float(r["Counter_Value"]) * 1024.0
                a = acc.setdefault(nm, [0.0, 0, 0.0])
                a[0] += v
                a[1] += 1
                a[2] = max(a[2], v)
            return acc
        fe, wr = per_kernel(fetch_csv), per_kernel(write_csv)
        # the calibration copy is the largest single dispatch of a copy kernel
        copy = max((nm for nm in fe if "copy" in nm.lower()), key=lambda nm: fe[nm][2])
        f_fac = (8 * COPY_DOUBLES) / fe[copy][2]
        w_fac = (8 * COPY_DOUBLES) / wr[copy][2]
        out += ["# HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
                f"Command (once per counter): `{pmc_command}`", "",
                f"Calibration: the 1 GiB device copy (`{copy[:60]}`) read FETCH_SIZE "
                f"{fe[copy][2] / 2**30:.3f} GiB and WRITE_SIZE {wr[copy][2] / 2**30:.3f} GiB; "
                f"scale factors {f_fac:.3f} (fetch), {w_fac:.3f} (write).", "",
                "| kernel | dispatches | read GB / dispatch | written GB / dispatch | total GB |",
                "|---|---|---|---|---|"]
        def short_name(nm):
            return nm.replace("kth::(anonymous namespace)::", "").replace("void ", "").split("(")[0]

        def base_name(nm):
            return short_name(nm).split("<")[0].split("::")[-1]

        keys = sorted((nm for nm in fe if "kth::" in nm), key=lambda nm: -fe[nm][0])
        for nm in keys:
            rf = fe[nm][0] * f_fac / fe[nm][1]
            rw = wr.get(nm, [0.0, 1])[0] * w_fac / max(wr.get(nm, [0.0, 1])[1], 1)
            short = short_name(nm)
            out.append(f"| `{short}` | {fe[nm][1]} | {rf / 1e9:.4f} | {rw / 1e9:.4f} | "
                       f"{(rf + rw) * fe[nm][1] / 1e9:.2f} |")
        # the four solves of the sample (one warm-up + three timed) and its six SpMV
        solve_k = ("k_gather", "k_solve_fwd", "k_lfwd_init", "k_lfwd_step", "k_lfwd_l21",
                   "k_lfwd_l21_reduce", "k_solve_bwd", "k_lbwd_l21", "k_lbwd_l21_reduce",
                   "k_lbwd_push", "k_scatter")
        tot = lambda nm: fe[nm][0] * f_fac + wr.get(nm, [0.0, 1])[0] * w_fac
        sv = [nm for nm in keys if base_name(nm) in solve_k]
        if sv:
            out += ["", f"- solve_hbm_bytes_per_solve: {sum(tot(nm) for nm in sv) / 4:.6e}",
                    "- solve_kernels: " + ", ".join(sorted({base_name(nm) for nm in sv}))]
        sp = [nm for nm in keys if base_name(nm) == "k_spmv2"]
        if sp:
            out += [f"- spmv_hbm_bytes_per_dispatch: {sum(tot(nm) for nm in sp) / sum(fe[nm][1] for nm in sp):.6e}"
                    f" (average of B x and the fused A x, B x)"]
        # the update products: k_gemm_lt (left-looking, small contribution blocks)
        # and k_gemm_cb128 (contribution blocks on 128 x 128 tiles), FP64
        sch = [nm for nm in keys if "k_gemm_lt<256, double>" in nm or "k_gemm_cb128<256, double>" in nm]
        if sch:
            launches = sum(fe[nm][1] for nm in sch)
            per = sum(tot(nm) for nm in sch) / launches
            out += ["", f"- k_gemm_lt_hbm_bytes_per_launch: {per:.6e}",
                    f"- k_gemm_lt_launches: {launches}",
                    "- (k_gemm_lt and k_gemm_cb128 together: "
                    + ", ".join(f"{base_name(nm)} {fe[nm][1]} launches, {tot(nm) / fe[nm][1]:.4e} B each"
                                for nm in sch) + ")",
                    f"- kernel_source_sha256: `{kernel_source_hash()}`"]
        out.append("")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n524k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--m-max", type=int, default=0,
                    help="stage-2 stopping count (0: chosen by the library's cost model)")
    ap.add_argument("--root-finder", type=int, default=1, choices=[0, 1],
                    help="stage 2: 0 bisection (Alg. 1'), 1 safeguarded interpolation")
    ap.add_argument("--b-solver", type=int, default=1, choices=[0, 1],
                    help="stage-1 B-solves: 0 LDL^T factor of B, 1 Jacobi CG when B is "
                         "strictly diagonally dominant")
    ap.add_argument("--skip", nargs="*", default=[],
                    choices=["stage2_other", "b_other", "hbm", "fp32_ir", "c3a", "c3b"],
                    help="extra legs to leave out")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="one factorization + a 1 GiB calibration copy, for rocprofv3 --pmc")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="print the markdown summary of rocprofv3 CSVs ('-' to skip one)")
    ap.add_argument("--summary-command", default="")
    ap.add_argument("--summary-pmc-command", default="")
    args = ap.parse_args()
    if args.summarize:
        st, fe, wr = (None if a == "-" else a for a in args.summarize)
        summarize(st, fe, wr, args.summary_command, args.summary_pmc_command)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (no path across GPUs is built); "
                                   "--gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.pmc_sample:
        pmc_sample()
        return

    import torch
    import pencilgen as pg
    import paper_1710_05134_amd as K

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    p = pg.workload(args.workload)
    log(f"workload {args.workload}: n={p.n} nnz={p.nnz} k={p.k}")
    ctx = K.Context(0, hip_stream=stream.cuda_stream)
    t0 = time.perf_counter()
    P = K.Pencil.from_pencilgen(ctx, p)
    t_cold = time.perf_counter() - t0
    ana = K.kth_analyze(p.rowptr, p.col)
    log(f"pencil ready in {t_cold:.2f} s (analysis flops {ana['flops']:.3e}, max front {ana['max_front']:.0f})")
    opts = K.default_opts(start_vectors=pg.start_vectors(p.n), root_finder=args.root_finder,
                          m_max=args.m_max, b_solver=args.b_solver)

    for w in range(args.warmup):
        lam, _, info = P.eig(p.k, opts=opts, want_x=False)
        log(f"warmup {w}: lambda={lam!r} validated={info['k_validated']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s in range(args.steps):
        lam, _, info = P.eig(p.k, opts=opts, want_x=False)
        infos.append(info)
        log(f"step {s}: lambda={lam!r} validated={info['k_validated']} "
            f"factorizations={info['n_factorizations']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sec = dt / args.steps
    info = infos[-1]

    # LDL^T rate and the roofline of the update products at the first bisection shift
    sigma2 = info["sigmas"][info["stage1_steps"]]
    profs = [P.profile_factor(sigma2) for _ in range(args.profile_reps)]
    tot = statistics.median(pr["total_s"] for pr in profs)
    # the LDL^T rate without per-launch events: factorizations at the same shift
    # through the pencil's inertia factor (one 64-byte readback each), median of the
    # same number of repetitions
    walls = []
    for _ in range(args.profile_reps):
        torch.cuda.synchronize()
        t_f = time.perf_counter()
        P.inertia(sigma2)
        walls.append(time.perf_counter() - t_f)
    tot_plain = statistics.median(walls)
    ldlt_gflops = ana["flops"] / tot_plain / 1e9
    classes = ("small", "assemble", "tile", "trsm", "gemm", "reduce")
    gm_s = statistics.median(pr["gemm"]["seconds"] for pr in profs)
    gm = profs[0]["gemm"]
    launches = max(gm["launches"], 1)
    per_launch_flops = gm["flops"] / launches
    per_launch_bytes = gm["bytes"] / launches
    avg_launch_s = gm_s / launches
    achieved = per_launch_flops / avg_launch_s / 1e12
    log(f"factorization {tot_plain * 1e3:.1f} ms = {ldlt_gflops:.0f} GFLOP/s ({tot * 1e3:.1f} ms with "
        f"events around every launch); k_gemm_lt {gm_s * 1e3:.1f} ms "
        f"over {gm['launches']} launches = {achieved:.2f} TFLOP/s, "
        f"{gm['bytes'] / gm_s / 1e9:.0f} GB/s algorithmic; classes "
        + ", ".join(f"{k} {statistics.median(pr[k]['seconds'] for pr in profs) * 1e3:.1f} ms"
                    for k in classes))
    cb_s = statistics.median(pr["gemm_cb"]["seconds"] for pr in profs)
    cb = profs[0]["gemm_cb"]
    ll_s = gm_s - cb_s
    log(f"  contribution blocks {cb_s * 1e3:.1f} ms in {cb['launches']} launches = "
        f"{cb['flops'] / max(cb_s, 1e-12) / 1e12:.2f} TFLOP/s; left-looking "
        f"{ll_s * 1e3:.1f} ms = {(gm['flops'] - cb['flops']) / max(ll_s, 1e-12) / 1e12:.2f} TFLOP/s")

    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"diamond tight-binding supercell {p.name} (n={p.n}, nnz={p.nnz}, k={p.k}, seed 0)",
            "n": p.n, "k": p.k,
            "lambda_k": lam, "k_validated": info["k_validated"],
            "rel_residual_normA": info["rel_residual_normA"],
            "factorizations_per_step": info["n_factorizations"],
            "stage1_steps": info["stage1_steps"], "bisection_steps": info["bisection_steps"],
            "si_steps": info["si_steps"],
            "m_max_used": info["m_max_used"],
            "b_solver": "Jacobi-preconditioned CG on B (b_solver=1)" if info["b_cg_iterations"] else
                        "LDL^T factor of B",
            "b_cg_iterations": info["b_cg_iterations"],
            "stage2": "bisection (Alg. 1')" if args.root_finder == 0 else
                      "safeguarded interpolation of the count (root_finder=1)",
            "min_pivot_rel": info["min_pivot_rel"], "max_abs_l": info["max_abs_l"],
            "weak_pivot_nudges": info["weak_pivot_nudges"],
            "t_task_s": info["t_task"][1:],
            "cold_pencil_create_s": t_cold,
            "ldlt_flops": ana["flops"],
            "ldlt_seconds": tot_plain,
            "ldlt_seconds_of": f"median of {args.profile_reps} factorizations (kth_inertia, wall time)",
            "ldlt_seconds_event_timed": tot,
            "ldlt_gflops": ldlt_gflops,
            "ldlt_frac_fp64_peak": ldlt_gflops / (PEAK_FP64_TFLOPS * 1e3),
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "update products: k_gemm_lt (left-looking, contribution blocks below 384 rows) "
                      "and k_gemm_cb128 (contribution blocks on 128x128 tiles), FP64 v_mfma_f64_16x16x4",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": gemm_traffic(),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "algorithmic_gbs": per_launch_bytes / avg_launch_s / 1e9,
            "launches": gm["launches"],
            "flops_per_launch": per_launch_flops,
            "avg_launch_us": avg_launch_s * 1e6,
            "classes_ms": {k: statistics.median(pr[k]["seconds"] for pr in profs) * 1e3 for k in classes},
            "gemm_split": {"contribution_blocks_ms": cb_s * 1e3,
                           "contribution_blocks_tflops": cb["flops"] / max(cb_s, 1e-12) / 1e12,
                           "left_looking_ms": ll_s * 1e3,
                           "left_looking_tflops": (gm["flops"] - cb["flops"]) / max(ll_s, 1e-12) / 1e12},
        },
    }

    def leg(name, fn):
        if name in args.skip:
            return
        t = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as e:            # report, keep the headline line
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"{name}: {time.perf_counter() - t:.1f} s: {json.dumps(out[name])[:300]}")

    def hbm_leg():
        # bandwidth of the solve and the SpMV at the shift-and-invert shift
        F = P.factor(info["sigma_si"])
        pr = F.profile_solve(10)
        F.close()
        return {
            "solve": {"seconds": pr["solve_s"], "bytes": pr["solve_bytes"],
                      "gbs": pr["solve_bytes"] / pr["solve_s"] / 1e9,
                      "frac": pr["solve_bytes"] / pr["solve_s"] / 1e9 / PEAK_HBM_GBS},
            "spmv_b": {"seconds": pr["spmv_b_s"], "bytes": pr["spmv_b_bytes"],
                       "gbs": pr["spmv_b_bytes"] / pr["spmv_b_s"] / 1e9,
                       "frac": pr["spmv_b_bytes"] / pr["spmv_b_s"] / 1e9 / PEAK_HBM_GBS},
            "spmv_ab": {"seconds": pr["spmv_ab_s"], "bytes": pr["spmv_ab_bytes"],
                        "gbs": pr["spmv_ab_bytes"] / pr["spmv_ab_s"] / 1e9,
                        "frac": pr["spmv_ab_bytes"] / pr["spmv_ab_s"] / 1e9 / PEAK_HBM_GBS},
            "peak_gbs": PEAK_HBM_GBS,
            "bytes_are": "algorithmic (one read of the factor per sweep; CSR values, indices, vectors once)",
        }

    def stage2_leg():
        # the same run with the other stage-2 rule
        other = 1 - args.root_finder
        oo = K.default_opts(start_vectors=pg.start_vectors(p.n), root_finder=other,
                            m_max=20 if other == 0 else args.m_max, b_solver=args.b_solver)
        P.eig(p.k, opts=oo, want_x=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lo, _, io = P.eig(p.k, opts=oo, want_x=False)
        torch.cuda.synchronize()
        return {"root_finder": other, "m_max": oo.m_max, "time_s": time.perf_counter() - t, "lambda_k": lo,
                "abs_diff": abs(lo - lam), "k_validated": io["k_validated"],
                "factorizations": io["n_factorizations"], "stage2_steps": io["bisection_steps"],
                "t_stage2_s": io["t_task"][4]}

    def b_leg():
        # the same run with the other stage-1 B-solve
        ob = K.default_opts(start_vectors=pg.start_vectors(p.n), root_finder=args.root_finder,
                            m_max=args.m_max, b_solver=1 - args.b_solver)
        P.eig(p.k, opts=ob, want_x=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lb, _, ib = P.eig(p.k, opts=ob, want_x=False)
        torch.cuda.synchronize()
        return {"b_solver": 1 - args.b_solver, "time_s": time.perf_counter() - t, "lambda_k": lb,
                "abs_diff": abs(lb - lam), "k_validated": ib["k_validated"],
                "factorizations": ib["n_factorizations"], "b_cg_iterations": ib["b_cg_iterations"],
                "t_b_factor_s": ib["t_task"][1]}

    def fp32_leg():
        # the same run with the shift-and-invert factor in FP32 + FP64 refinement
        o32 = K.default_opts(start_vectors=pg.start_vectors(p.n), si_precision=K.KTH_FP32_IR,
                             root_finder=args.root_finder, m_max=args.m_max, b_solver=args.b_solver)
        P.eig(p.k, opts=o32, want_x=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        l32, _, i32 = P.eig(p.k, opts=o32, want_x=False)
        torch.cuda.synchronize()
        return {"time_s": time.perf_counter() - t, "lambda_k": l32, "abs_diff_vs_fp64": abs(l32 - lam),
                "k_validated": i32["k_validated"], "rel_residual_normA": i32["rel_residual_normA"],
                "si_steps": i32["si_steps"], "ir_steps": i32["ir_steps"],
                "ir_fallback": i32["ir_fallback"], "t_si_factor_s": i32["t_task"][5],
                "t_si_lanczos_s": i32["t_task"][6], "fp64_t_si_lanczos_s": info["t_task"][6]}

    def c3a_leg():
        # 64 shifts of the n = 131072 pencil per round, against one at a time and
        # against sequential bisection to the same stopping rule
        q = pg.workload("n131k")
        Q = K.Pencil.from_pencilgen(ctx, q)
        oq = K.default_opts(start_vectors=pg.start_vectors(q.n))
        _, _, iq = Q.eig(q.k, opts=oq, want_x=False)
        s1 = iq["stage1_steps"]
        sl, su = sorted(iq["sigmas"][s1 - 2:s1]) if s1 >= 2 else (iq["sigma_lower"], iq["sigma_upper"])
        sig = [sl + (su - sl) * (i + 1) / 65.0 for i in range(64)]
        Q.inertia_batch(sig[:2])
        torch.cuda.synchronize()
        t = time.perf_counter()
        nb = Q.inertia_batch(sig)
        t_batch = time.perf_counter() - t
        t = time.perf_counter()
        ns_ = [Q.nu(x) for x in sig]
        t_single = time.perf_counter() - t
        om = K.default_opts(start_vectors=pg.start_vectors(q.n), multisection=64)
        Q.eig(q.k, opts=om, want_x=False)
        t = time.perf_counter()
        lm, _, im = Q.eig(q.k, opts=om, want_x=False)
        t_ms_eig = time.perf_counter() - t
        t = time.perf_counter()
        l1, _, i1 = Q.eig(q.k, opts=oq, want_x=False)
        t_bi_eig = time.perf_counter() - t
        return {"workload": "n131k (n=131072), 64 equispaced interior shifts of the stage-1 interval",
                "round_64_batched_s": t_batch, "round_64_one_at_a_time_s": t_single,
                "counts_equal": list(map(int, nb)) == ns_,
                "stage2_multisection64_s": im["t_task"][4], "stage2_rounds": im["bisection_steps"],
                "stage2_bisection_s": i1["t_task"][4], "bisection_steps": i1["bisection_steps"],
                "eig_multisection64_s": t_ms_eig, "eig_bisection_s": t_bi_eig,
                "lambda_abs_diff": abs(lm - l1), "validated": im["k_validated"] == i1["k_validated"] == q.k}

    def c3b_leg():
        # 256 uneven pencils (n in [500, 8000]) in one batched call, against a loop
        pens = pg.uneven_batch(count=256, seed=0)
        t = time.perf_counter()
        Ps = [K.Pencil.from_pencilgen(ctx, q) for q in pens]
        t_create = time.perf_counter() - t
        ks = [q.k for q in pens]
        K.eig_batch(ctx, Ps[:8], ks[:8], want_x=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = K.eig_batch(ctx, Ps, ks, want_x=False)
        t_batch = time.perf_counter() - t
        t = time.perf_counter()
        loop = [Pq.eig(kq, want_x=False)[0] for Pq, kq in zip(Ps, ks)]
        t_loop = time.perf_counter() - t
        ok = sum(r[0] == K.KTH_OK and r[3]["k_validated"] == kq for r, kq in zip(res, ks))
        same = sum(r[1] == lq for r, lq in zip(res, loop))
        for Pq in Ps:
            Pq.close()
        return {"pencils": len(pens), "n_range": [min(q.n for q in pens), max(q.n for q in pens)],
                "batched_s": t_batch, "pencils_per_s": len(pens) / t_batch,
                "loop_of_kth_eig_s": t_loop, "loop_pencils_per_s": len(pens) / t_loop,
                "speedup": t_loop / t_batch, "validated": ok, "lambda_equal_to_loop": same,
                "host_analysis_s": t_create,
                "factorizations": sum(r[3]["n_factorizations"] for r in res)}

    leg("stage2_other", stage2_leg)
    leg("b_other", b_leg)
    leg("hbm", hbm_leg)
    leg("fp32_ir", fp32_leg)
    leg("c3a", c3a_leg)
    leg("c3b", c3b_leg)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)...")
        out["cpu_baseline"] = cpu_baseline(p, info["n_factorizations"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
