#!/usr/bin/env python3
"""Throughput of the randomized preconditioned Newton solver on one MI355X.

A step is one complete Newton solve from the zero guess: assembly with the row
scale, sketch, QR, preconditioned LSQR, back-transform, line search and update,
repeated until the stop test fires.  The workload is the steady 3-D Gray-Scott
system on the unit cube, 4 x 4 x 4 boxes, 300 tanh features per box and
component (n = 38,400 unknowns), 10^3 collocation points per box and 10 x 10 face
grids (m = 204,800 rows), sketch s = 2n, LSQR tolerance 1e-10.

The timed solver is the mixed-precision form by default: the sketch on the BF16
matrix cores (error-free fixed-point pieces, FP64 chunk sums), LSQR products on
an FP32 copy of D J (falling back to FP64 if a step stalls), QR, triangular
solves, residuals and the update in FP64.  The plain FP64 solver is timed after
it on the same problem (one solve) for comparison.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sketch-prec bf16|fp8|f64] [--lsqr-prec f32|f64]

prints one JSON line.  The problem description is uploaded before the timed
region; the coefficient vector lives in device memory.  Kernel times for the
roofline figures are HIP events recorded by the library around its kernels on
the stream they run on, over the timed steps.

    python bench.py --summarize-rocpd DB

prints a per-kernel summary (launches, total and average duration) of a
rocprofv3 kernel-trace database.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sqlite3
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix
PEAK_FP8_TFLOPS = 5000.0     # MI355X dense FP8 matrix
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PREC = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}

# HBM bytes per launch of the QR's trailing-update products on the Gray-Scott workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch, scaled by 2.0 and 1.0: what the
# same counters read for an elementwise copy of 1 GiB); valid only while the kernels are unchanged,
# so a kernel without counters taken on its current code reports null
TRAFFIC_BYTES = {
    "qr_gemm_tn": (6439910.3 * 2.0 + 276686.2 * 1.0) * 1024.0,
    "qr_gemm_nn": (6164443.1 * 2.0 + 4851457.7 * 1.0) * 1024.0,
}

METRIC = "Newton solves/s at relL2<=1e-6; sketch-GEMM TFLOP/s; LSQR SpMV HBM GB/s"


def summarize_rocpd(db_path: str) -> str:
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    iname = cols.index("name") if "name" in cols else cols.index("kernel_name")
    ist, ien = cols.index("start"), cols.index("end")
    agg = {}
    for r in cur.execute("select * from kernels"):
        n = r[iname].replace("(anonymous namespace)::", "")
        n = re.sub(r"\(.*", "", n)
        d = (r[ien] - r[ist]) * 1e-9
        a = agg.setdefault(n, [0, 0.0])
        a[0] += 1
        a[1] += d
    tot = sum(v[1] for v in agg.values())
    lines = [f"# kernel summary of {os.path.basename(db_path)}: {sum(v[0] for v in agg.values())} dispatches, "
             f"{tot:.4f} s of kernel time",
             f"{'total_s':>10} {'pct':>6} {'calls':>7} {'avg_us':>12}  kernel"]
    for n, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{t:10.4f} {100 * t / tot:6.1f} {c:7d} {1e6 * t / c:12.1f}  {n}")
    return "\n".join(lines)


def cpu_baseline(quick: bool) -> dict:
    """The CPU oracle on a bounded sample of the same workload family."""
    import numpy as np
    import rfm_workloads as W
    from oracle import rfm as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    nsub, J, q = ((2, 1, 1), 30, 4) if quick else ((2, 2, 2), 200, 7)
    prob = W.config2(nsub=nsub, J=J, q=q, test_per_dim=2)
    t0 = time.perf_counter()
    u, st = O.ipn(prob, opts=O.Opts(gamma=2.0, lsqr_tol=1e-10))
    dt = time.perf_counter() - t0
    n_full = 4 * 4 * 4 * 2 * 300
    scale = (n_full / prob.n) ** 3
    return {"value": 1.0 / (dt * scale), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle IPN (FP64 numpy, dense J, Philox sketch, LAPACK QR, own LSQR) on the same "
                       f"Gray-Scott system with {nsub} boxes, J={J}, q={q} (n={prob.n}, m={O.row_table(prob)[1]}): "
                       f"{dt:.2f} s for {st.outer_iters} Newton steps; extrapolated to n={n_full} by (n/n_s)^3, "
                       f"the growth of the QR that dominates the solve"),
            "measured_s": dt, "n_sample": prob.n}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["gray-scott", "allen-cahn-hole", "helmholtz-cosh", "helmholtz-holes"],
                    default="gray-scott",
                    help="allen-cahn-hole: space-time Allen-Cahn around a moving disc, 4 x 4 x 8 boxes, "
                         "J = 400, q = 12 (n = 51,200); helmholtz-cosh: Lap u - 100 u + 10 cosh(u) = f on the "
                         "unit cube, 2 x 2 x 2 boxes, --features J, --points q; helmholtz-holes: -Lap u - 64 u "
                         "+ u^3 = f on the unit cube minus four spheres, --boxes per axis (8: n = 128,000, "
                         "the sketch streamed), J = 250, q = 8; none of them runs the warm-start study or the "
                         "CPU baseline")
    ap.add_argument("--features", type=int, default=400, help="helmholtz-cosh: J per box")
    ap.add_argument("--points", type=int, default=20, help="helmholtz-cosh: q (q^3 points per box)")
    ap.add_argument("--boxes", type=int, default=8, help="helmholtz-holes: boxes per axis")
    ap.add_argument("--rows-per-pass", type=int, default=0,
                    help="sketch rows per pass of the streamed QR (0: stream only when B does not fit)")
    ap.add_argument("--verbose", action="store_true", help="progress lines from the solver on stderr")
    ap.add_argument("--method", choices=["ipn", "amipn"], default="ipn")
    ap.add_argument("--sketch-prec", choices=["bf16", "fp8", "f64"], default="bf16")
    ap.add_argument("--sketch-kind", choices=["gaussian", "count"], default="gaussian",
                    help="count: the paper's count sketch (FP64; implies --sketch-prec f64)")
    ap.add_argument("--lsqr-prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-warm-start-study", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-rocpd", metavar="DB")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the solves, copy a buffer of this many MiB three times (a reference "
                         "kernel of known traffic for scaling hardware byte counters)")
    a = ap.parse_args()
    if a.summarize_rocpd:
        print(summarize_rocpd(a.summarize_rocpd))
        return
    if a.gpus != 1:
        print(f"bench.py: a solve runs on one GPU; --gpus {a.gpus} is not supported "
              f"(independent solves, one process per GPU, are how more GPUs are used)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import rfm_workloads as W
    import paper_2510_04170_amd as R

    rank = int(os.environ.get("RANK", "0"))
    if a.workload == "allen-cahn-hole":
        a.no_warm_start_study = True
        a.no_cpu_baseline = True
        prob = W.config4()
        workload = "allen_cahn_space_time_moving_hole_4x4x8_J400_q12"
    elif a.workload == "helmholtz-holes":
        a.no_warm_start_study = True
        a.no_cpu_baseline = True
        prob = W.config3(nsub=(a.boxes,) * 3)
        workload = f"helmholtz_3d_4_holes_{a.boxes}x{a.boxes}x{a.boxes}_J250_q8"
    elif a.workload == "helmholtz-cosh":
        a.no_warm_start_study = True
        a.no_cpu_baseline = True
        prob = W.helmholtz_cosh(nsub=(2, 2, 2), J=a.features, q=a.points)
        workload = f"helmholtz_cosh_3d_2x2x2_J{a.features}_q{a.points}"
    else:
        prob = W.config2()
        workload = "gray_scott_3d_4x4x4_J300_q10"
    t_setup = time.perf_counter()
    lp = R.from_description(prob)
    print(f"[bench] problem uploaded in {time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
    n, m = lp.n, lp.m
    method = R.RFM_AMIPN if a.method == "amipn" else R.RFM_IPN
    if a.sketch_kind == "count":
        a.sketch_prec = "f64"
    opts = R.default_opts(method=method, sketch_factor=2.0, lsqr_tol=1e-10, m_max=5,
                          sketch_prec=PREC[a.sketch_prec], lsqr_prec=PREC[a.lsqr_prec],
                          sketch_kind=R.RFM_SKETCH_COUNT if a.sketch_kind == "count" else R.RFM_SKETCH_GAUSSIAN,
                          sketch_rows_per_pass=a.rows_per_pass, verbose=int(a.verbose))
    opts64 = R.default_opts(method=method, sketch_factor=2.0, lsqr_tol=1e-10, m_max=5,
                            sketch_rows_per_pass=a.rows_per_pass, verbose=int(a.verbose))
    dev = torch.device("cuda", 0)
    u = torch.zeros(n, dtype=torch.float64, device=dev)
    print(f"[bench] workload ready: m={m} n={n}; warmup {a.warmup}", file=sys.stderr, flush=True)
    if a.copy_calibration_mib > 0:
        nb = a.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 elementwise copies of {nb} bytes (read {nb}, write {nb} each)",
              file=sys.stderr, flush=True)
        del src, dst
    for _ in range(a.warmup):
        u.zero_()
        lp.solve(u, opts)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    lp.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for k in range(a.steps):
        u.zero_()
        _, stats, rc = lp.solve(u, opts)
        print(f"[bench] step {k + 1}/{a.steps}: status {rc}, IT {stats['outer_iters']}, NJ {stats['jac_evals']}, "
              f"{stats['t_total']:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = lp.profile_read()
    lp.profile_enable(False)

    elapsed = t1 - t0
    val = lp.eval(u, prob.test_x, prob.test_owner)
    ex = prob.exact(prob.test_x)
    rel = (np.linalg.norm(val - ex, axis=0) / np.linalg.norm(ex, axis=0)).tolist()

    ref64 = None
    if not a.no_fp64_reference and (a.sketch_prec != "f64" or a.lsqr_prec != "f64" or a.sketch_kind == "count"):
        # the plain FP64 solver on the same problem, for the throughput ratio and the field difference
        u64 = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, st64, rc64 = lp.solve(u64, opts64)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(f"[bench] FP64 reference solve: status {rc64}, IT {st64['outer_iters']}, {t3 - t2:.2f} s",
              file=sys.stderr, flush=True)
        v64 = lp.eval(u64, prob.test_x, prob.test_owner)
        rel64 = (np.linalg.norm(v64 - ex, axis=0) / np.linalg.norm(ex, axis=0)).tolist()
        ref64 = {"solves_per_s": 1.0 / (t3 - t2), "s_per_solve": t3 - t2, "status": rc64,
                 "outer_iters": st64["outer_iters"], "lsqr_iters": st64["lsqr_iters"], "relL2": rel64,
                 "field_diff_vs_mixed": float(np.linalg.norm(val - v64) / np.linalg.norm(v64)),
                 "speedup_of_mixed": (t3 - t2) / (elapsed / a.steps)}

    sk_name = "sketch_count" if a.sketch_kind == "count" else \
        {"f64": "sketch_f64", "bf16": "sketch_bf16", "fp8": "sketch_fp8"}[a.sketch_prec]
    sk_peak = {"f64": PEAK_FP64_TFLOPS, "bf16": PEAK_BF16_TFLOPS, "fp8": PEAK_FP8_TFLOPS}[a.sketch_prec]

    def rate(name, what):
        k = kern.get(name)
        if not k or k["seconds"] <= 0:
            return None
        return (k["flops"] / k["seconds"] / 1e12) if what == "flops" else (k["bytes"] / k["seconds"] / 1e9)

    kernels = {}
    for name, k in kern.items():
        kernels[name] = {"launches": k["launches"], "seconds": round(k["seconds"], 6),
                         "avg_us": round(1e6 * k["seconds"] / max(1, k["launches"]), 2)}
        if k["flops"] > 0:
            kernels[name]["tflops"] = round(k["flops"] / k["seconds"] / 1e12, 3)
        if k["bytes"] > 0:
            kernels[name]["gbs"] = round(k["bytes"] / k["seconds"] / 1e9, 1)
    cand = {nm: k for nm, k in kern.items() if not nm.endswith("_total")}
    dom = max(cand, key=lambda nm: cand[nm]["seconds"])
    dk = cand[dom]
    mfma_bound = dk["flops"] > 0 and dk["flops"] / max(dk["bytes"], 1.0) > PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    if mfma_bound:
        achieved = dk["flops"] / dk["seconds"] / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": TRAFFIC_BYTES.get(dom) if a.workload == "gray-scott" else None,
                "per_launch_alg_bytes": dk["bytes"] / dk["launches"],
                "per_launch_flops": dk["flops"] / dk["launches"],
                "avg_launch_us": round(1e6 * dk["seconds"] / dk["launches"], 2)}
    else:
        achieved = dk["bytes"] / dk["seconds"] / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "per_launch_bytes": dk["bytes"] / dk["launches"],
                "avg_launch_us": round(1e6 * dk["seconds"] / dk["launches"], 2)}

    dtype = "f64" if (a.sketch_prec, a.lsqr_prec) == ("f64", "f64") else \
        f"f64 QR/TRSV/residual; {a.sketch_prec} sketch; {a.lsqr_prec} LSQR operator"
    sk = rate(sk_name, "flops")
    out = {
        "metric": METRIC,
        "value": a.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "m": m, "s": 2 * n, "method": a.method,
                   "sketch": ("count_sketch_philox4x64_f64" if a.sketch_kind == "count" else
                              "gaussian_philox4x64_f64" if a.sketch_prec == "f64" else
                              f"philox4x64_code_table_{a.sketch_prec}_exact_pieces"),
                   "sketch_prec": a.sketch_prec, "lsqr_prec": a.lsqr_prec, "lsqr_tol": 1e-10, "outer_tol": 1e-10,
                   "row_scale_c": 100.0, "initial_guess": "zero"},
        "relL2": rel,
        "relL2_target_met": bool(max(rel) <= 1e-6),
        "newton": {"outer_iters": stats["outer_iters"], "jac_evals": stats["jac_evals"],
                   "lsqr_iters": stats["lsqr_iters"], "final_resnorm": stats["final_resnorm"],
                   "status": stats["status"], "lsqr_fp64_fallback": stats["lsqr_fp64_fallback"]},
        "sketch_tflops": sk,
        "sketch_frac_of_peak": None if sk is None else sk / sk_peak,
        "sketch_peak_tflops": sk_peak,
        "lsqr_spmv_gbs": {k: rate(k, "bytes") for k in ("jmul", "jtmul", "jmul_f32", "jtmul_f32") if k in kern},
        "fp64_path": ref64,
        "roofline": roof,
        "kernels": kernels,
    }
    if not a.no_warm_start_study:
        # learned initial guess on a small member family of the same system (the full-size
        # family would need hundreds of full-size training solves): Newton steps and time
        # against the zero guess on held-out members, the FP64 solver deciding the answer
        from paper_2510_04170_amd import warmstart as WS
        print("[bench] warm-start study ...", file=sys.stderr, flush=True)
        ws = WS.run(n_train=48, n_test=4)
        out["warm_start"] = {"family": ws["family"], "network": ws["network"], "seconds": ws["seconds"],
                             "mean": ws["mean"],
                             "max_field_diff_vs_zero_guess": max(r["field_diff"] for r in ws["per_draw"]),
                             "kept": [r["warm"]["kept"] for r in ws["per_draw"]]}
    if rank == 0 and not a.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.quick_cpu_baseline)
    if rank == 0:
        print(json.dumps(out))


if __name__ == "__main__":
    main()
