#!/usr/bin/env python3
"""Throughput of the randomized preconditioned Newton solver on one MI355X.

A step is one complete Newton solve from the zero guess: assembly with the row
scale, sketch, QR, preconditioned LSQR, back-transform, line search and update,
repeated until the stop test fires.  The workload is the steady 3-D Gray-Scott
system on the unit cube, 4 x 4 x 4 boxes, 300 tanh features per box and
component (n = 38,400 unknowns), 10^3 collocation points per box and 10 x 10 face
grids (m = 204,800 rows), sketch s = 2n, LSQR tolerance 1e-10.

The timed solver (`value`) is the plain FP64 form, the paper's arithmetic: FP64
Gaussian sketch on the FP64 matrix cores, FP64 QR, LSQR on the FP64 Jacobian,
FP64 triangular solves, residuals, line search and update.  The mixed-precision
form (the sketch on the BF16 matrix cores as error-free fixed-point pieces with
FP64 chunk sums, LSQR products on an FP32 copy of D J, everything else in FP64)
is timed after it on the same problem (`mixed_form`: its time per solve, its
speedup over the FP64 form and the difference of the two fields).  The metric
asks for solves that reach relL2 <= 1e-6; on this workload no coefficient
vector of the stated features gets there (the best fit of u*, v* on the test
points is 6.3e-6 and 1.3e-5), so `relL2` and `relL2_target_met` say what the
solves reach.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form f64|mixed] [--other-steps N]

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

# HBM bytes per launch on the Gray-Scott workload, from two rocprofv3 --pmc runs of
# `bench.py --profile-stages 1 --copy-calibration-mib 1024` (FETCH_SIZE, WRITE_SIZE in KiB per dispatch,
# scaled by 2.0 and 1.0: what the same counters read for an elementwise copy of 1 GiB; FETCH_SIZE counts a
# 128-byte read request as 64 bytes here, and the read-request counters by size agree with the scaled
# figure within 0.5% for the products and the triangular solves).  A library stage spanning two kernels
# (J^T y: tile products, then their reduction) adds both.  Valid only while the kernels are unchanged, so
# a kernel without counters taken on its current code reports null.
TRAFFIC_BYTES = {
    "qr_gemm_tn": (6309084.9 * 2.0 + 276686.2 * 1.0) * 1024.0,
    "qr_gemm_nn": (6164425.4 * 2.0 + 4851457.7 * 1.0) * 1024.0,
    "jmul": (411221.0 * 2.0 + 1525.9) * 1024.0,
    "jmul_f32": (207244.5 * 2.0 + 1525.1) * 1024.0,
    "jtmul": (441649.0 * 2.0 + 14187.7 + 8024.8 * 2.0 + 267.7) * 1024.0,
    "jtmul_f32": (232479.4 * 2.0 + 14187.9 + 8024.8 * 2.0 + 267.7) * 1024.0,
    "trsv": ((2576417.4 + 2581714.9) / 2 * 2.0 + (818.3 + 829.3) / 2) * 1024.0,
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


def summarize_counters(csv_path: str) -> str:
    """Per-kernel mean of each hardware counter per dispatch from a rocprofv3 --pmc counter_collection.csv."""
    import csv
    agg = {}
    with open(csv_path, newline="") as f:
        rows = csv.DictReader(f)
        cols = rows.fieldnames or []
        kcol = next(c for c in cols if c.lower() in ("kernel_name", "kernel-name", "name"))
        ncol = next(c for c in cols if c.lower() in ("counter_name", "counter-name"))
        vcol = next(c for c in cols if c.lower() in ("counter_value", "counter-value", "value"))
        dcol = next((c for c in cols if c.lower() in ("dispatch_id", "dispatch-id", "correlation_id")), None)
        for r in rows:
            k = re.sub(r"\(.*", "", r[kcol].replace("(anonymous namespace)::", ""))
            key = (k, r[ncol])
            a = agg.setdefault(key, [0.0, set()])
            a[0] += float(r[vcol])
            a[1].add(r[dcol] if dcol else len(a[1]))
    lines = [f"# counters of {os.path.basename(csv_path)}: mean per dispatch",
             f"{'dispatches':>10} {'mean':>16}  counter  kernel"]
    for (k, c), (tot, ds) in sorted(agg.items()):
        lines.append(f"{len(ds):10d} {tot / max(1, len(ds)):16.1f}  {c}  {k}")
    return "\n".join(lines)


def _host_info() -> dict:
    """CPU model, logical CPUs and RAM of the machine the CPU baseline runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_gib": ram}


def cpu_baseline(quick: bool) -> dict:
    """The CPU oracle (IPN, FP64, the same sketch / QR / LSQR / line search as the GPU path) on two bounded
    samples of the same workload family, extrapolated to the full size by (n / n_s)^3 (the QR's growth)."""
    import numpy as np
    import rfm_workloads as W
    from oracle import rfm as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    samples = [((2, 1, 1), 30, 4), ((2, 1, 1), 40, 4)] if quick else [((2, 2, 1), 200, 7), ((2, 2, 2), 200, 7)]
    n_full = 4 * 4 * 4 * 2 * 300
    runs = []
    for nsub, J, q in samples:
        prob = W.config2(nsub=nsub, J=J, q=q, test_per_dim=2)
        t0 = time.perf_counter()
        u, st = O.ipn(prob, opts=O.Opts(gamma=2.0, lsqr_tol=1e-10))
        dt = time.perf_counter() - t0
        runs.append({"boxes": list(nsub), "J": J, "q": q, "n": prob.n, "m": int(O.row_table(prob)[1]),
                     "seconds": round(dt, 3), "newton_steps": st.outer_iters,
                     "extrapolated_solves_per_s": 1.0 / (dt * (n_full / prob.n) ** 3)})
    big = runs[-1]
    return {"value": big["extrapolated_solves_per_s"], "unit": "solves/s", "cores": threads, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"oracle IPN (FP64 numpy, dense J, Philox Gaussian sketch, LAPACK QR, own LSQR) on the same "
                       f"Gray-Scott system at two reduced sizes (n = {runs[0]['n']} and {big['n']}); value from the "
                       f"larger ({big['seconds']:.1f} s for {big['newton_steps']} Newton steps) extrapolated to "
                       f"n = {n_full} by (n/n_s)^3, the growth of the QR that dominates the solve"),
            "samples": runs, "host": _host_info()}


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def profile_stages(lp, prob, reps: int) -> dict:
    """Each hot kernel of one Newton step on the workload, outside a solve, for kernel-level timing and
    hardware counters: assembly at a random iterate, the FP64 and the BF16 sketch, the QR, then `reps`
    LSQR solves (tolerance 1e-10) with the FP64 and with the FP32 copy of D J, each running its J x,
    J^T y and both triangular solves once per iteration."""
    import numpy as np
    rng = np.random.default_rng(11)
    u = 0.1 * rng.normal(size=lp.n)
    lp.profile_enable(True)
    lp.stage_assemble(u, 100.0)
    lp.stage_sketch(2.0, 1, 0, PREC["bf16"])
    lp.stage_sketch(2.0, 1, 0, PREC["f64"])
    lp.stage_qr()
    rhs = rng.normal(size=lp.m)
    iters = {}
    for prec in ("f64", "f32"):
        for _ in range(reps):
            _, it, _ = lp.stage_lsqr(rhs, 1e-10, 500, PREC[prec])
        iters[prec] = it
    kern = lp.profile_read()
    lp.profile_enable(False)
    out = {}
    for name, k in kern.items():
        rec = {"launches": k["launches"], "avg_us": 1e6 * k["seconds"] / max(1, k["launches"])}
        if k["flops"] > 0:
            rec["tflops"] = k["flops"] / k["seconds"] / 1e12
            rec["flops_per_launch"] = k["flops"] / k["launches"]
        if k["bytes"] > 0:
            rec["GB_s"] = k["bytes"] / k["seconds"] / 1e9
            rec["bytes_per_launch"] = k["bytes"] / k["launches"]
        out[name] = rec
    return {"stages": out, "lsqr_iters": iters, "reps": reps}


def pieces_study(lp, prec: str, pieces_list) -> dict:
    """How many fixed-point pieces of D J the low-precision sketch needs: for each piece count, the R of
    that sketch and the LSQR iterations it takes to solve min ||D J R^-1 y - b|| to 1e-10 for a random b
    (with the FP64 sketch's R for comparison).  LSQR's iterations grow with kappa(D J R^-1), about
    ln(1e-10) / ln((kappa - 1) / (kappa + 1)) for a well-spread spectrum, so the count whose iterations
    match the FP64 sketch's preconditions as well."""
    import numpy as np
    rng = np.random.default_rng(5)
    u = 0.1 * rng.normal(size=lp.n)
    lp.stage_assemble(u, 100.0)
    rhs = rng.normal(size=lp.m)
    rows = []
    for p in [0] + list(pieces_list):
        t0 = time.perf_counter()
        if p == 0:
            lp.stage_sketch(2.0, 1, 0, PREC["f64"])
        else:
            lp.stage_sketch(2.0, 1, 0, PREC[prec], p)
        lp.stage_qr()
        _, it, istop = lp.stage_lsqr(rhs, 1e-10, 500, PREC["f64"])
        rows.append({"pieces": p if p else "f64", "lsqr_iters": it, "istop": istop,
                     "seconds": round(time.perf_counter() - t0, 3)})
        print(f"[bench] pieces study {prec}: {rows[-1]}", file=sys.stderr, flush=True)
    return {"prec": prec, "rows": rows}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["gray-scott", "poisson-2d", "allen-cahn-hole", "helmholtz-cosh", "helmholtz-holes"],
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
    ap.add_argument("--form", choices=["f64", "mixed"], default="f64",
                    help="the timed form: f64 (the paper's arithmetic) or mixed (--sketch-prec, --lsqr-prec)")
    ap.add_argument("--other-steps", type=int, default=2,
                    help="timed solves of the other form after one untimed one (0: skip it)")
    ap.add_argument("--sketch-prec", choices=["bf16", "fp8"], default="bf16", help="the mixed form's sketch")
    ap.add_argument("--lsqr-prec", choices=["f32", "f64"], default="f32", help="the mixed form's LSQR operator")
    ap.add_argument("--sketch-kind", choices=["gaussian", "count"], default="gaussian",
                    help="count: the paper's count sketch in the FP64 form")
    ap.add_argument("--warm-train", type=int, default=512, help="warm-start study: training draws")
    ap.add_argument("--warm-test", type=int, default=128, help="warm-start study: held-out draws")
    ap.add_argument("--no-warm-start-study", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-rocpd", metavar="DB")
    ap.add_argument("--summarize-counters", metavar="CSV",
                    help="per-kernel mean counter values of a rocprofv3 --pmc counter_collection.csv")
    ap.add_argument("--pieces-study", action="store_true",
                    help="instead of timing solves: LSQR iterations with the R of the low-precision sketch "
                         "(--sketch-prec) at 1 .. 6 (BF16) or 2 .. 12 (FP8) pieces against the FP64 sketch's R")
    ap.add_argument("--profile-stages", type=int, default=0, metavar="REPS",
                    help="instead of timing solves: run each hot kernel of a Newton step on the workload once "
                         "(assembly, FP64 and BF16 sketch, QR) and REPS LSQR solves with the FP64 and the FP32 "
                         "operator, and print their kernel times (for rocprofv3 counter runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the solves, copy a buffer of this many MiB three times (a reference "
                         "kernel of known traffic for scaling hardware byte counters)")
    a = ap.parse_args()
    if a.summarize_rocpd:
        print(summarize_rocpd(a.summarize_rocpd))
        return
    if a.summarize_counters:
        print(summarize_counters(a.summarize_counters))
        return
    if a.gpus != 1:
        print(f"bench.py: a solve runs on one GPU and the benchmark measures one GPU; --gpus {a.gpus} is not "
              f"supported (independent solves, one process per GPU, are how more GPUs would be used)",
              file=sys.stderr)
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
    elif a.workload == "poisson-2d":
        a.no_warm_start_study = True
        a.no_cpu_baseline = True
        prob = W.config1()
        workload = "poisson_2d_cubic_2x2_J200_q20"
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
    n, m, nnz = lp.n, lp.m, lp.nnz
    s_rows = 2 * n
    if a.copy_calibration_mib > 0:
        dev = torch.device("cuda", 0)
        nb = a.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 elementwise copies of {nb} bytes (read {nb}, write {nb} each)",
              file=sys.stderr, flush=True)
        del src, dst
    if a.pieces_study:
        plist = range(1, 7) if a.sketch_prec == "bf16" else range(2, 13, 2)
        res = pieces_study(lp, a.sketch_prec, plist)
        lp.close()
        print(json.dumps({"workload": workload, "n": n, "m": m, **res}), flush=True)
        return
    if a.profile_stages > 0:
        res = profile_stages(lp, prob, a.profile_stages)
        lp.close()
        print(json.dumps({"workload": workload, "n": n, "m": m, "nnz_J": nnz, **res}), flush=True)
        return
    method = R.RFM_AMIPN if a.method == "amipn" else R.RFM_IPN
    common = dict(method=method, sketch_factor=2.0, lsqr_tol=1e-10, m_max=5, sketch_rows_per_pass=a.rows_per_pass,
                  verbose=int(a.verbose))
    opts_f64 = R.default_opts(sketch_kind=R.RFM_SKETCH_COUNT if a.sketch_kind == "count" else R.RFM_SKETCH_GAUSSIAN,
                              **common)
    opts_mixed = R.default_opts(sketch_prec=PREC[a.sketch_prec], lsqr_prec=PREC[a.lsqr_prec], **common)
    forms = {"f64": opts_f64, "mixed": opts_mixed}
    other = "mixed" if a.form == "f64" else "f64"
    dev = torch.device("cuda", 0)
    u = torch.zeros(n, dtype=torch.float64, device=dev)
    print(f"[bench] workload ready: m={m} n={n} nnz(J)={nnz}; timed form {a.form}; warmup {a.warmup}",
          file=sys.stderr, flush=True)
    for k in range(a.warmup):
        u.zero_()
        _, st, rc = lp.solve(u, forms[a.form])
        print(f"[bench] warmup {k + 1}/{a.warmup}: status {rc}, {st['t_total']:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    lp.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for k in range(a.steps):
        u.zero_()
        _, stats, rc = lp.solve(u, forms[a.form])
        print(f"[bench] step {k + 1}/{a.steps}: status {rc}, IT {stats['outer_iters']}, NJ {stats['jac_evals']}, "
              f"{stats['t_total']:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = lp.profile_read()
    lp.profile_enable(False)
    elapsed = t1 - t0

    ex = prob.exact(prob.test_x)
    val = lp.eval(u, prob.test_x, prob.test_owner)
    rel = (np.linalg.norm(val - ex, axis=0) / np.linalg.norm(ex, axis=0)).tolist()

    # the other form on the same problem: one untimed solve, then --other-steps timed ones
    other_out, kern_other = None, {}
    if a.other_steps > 0:
        u2 = torch.zeros(n, dtype=torch.float64, device=dev)
        lp.solve(u2, forms[other])
        lp.profile_enable(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k in range(a.other_steps):
            u2.zero_()
            _, st2, rc2 = lp.solve(u2, forms[other])
            print(f"[bench] {other} form {k + 1}/{a.other_steps}: status {rc2}, IT {st2['outer_iters']}, "
                  f"{st2['t_total']:.2f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        kern_other = lp.profile_read()
        lp.profile_enable(False)
        v2 = lp.eval(u2, prob.test_x, prob.test_owner)
        per_other = (t3 - t2) / a.other_steps
        per_main = elapsed / a.steps
        v_f64, v_mixed = (val, v2) if a.form == "f64" else (v2, val)
        other_out = {"form": other, "s_per_solve": per_other, "solves_per_s": 1.0 / per_other,
                     "steps": a.other_steps, "status": rc2, "outer_iters": st2["outer_iters"],
                     "jac_evals": st2["jac_evals"], "lsqr_iters": st2["lsqr_iters"],
                     "relL2": (np.linalg.norm(v2 - ex, axis=0) / np.linalg.norm(ex, axis=0)).tolist(),
                     "field_diff_mixed_vs_f64": _rel(v_mixed, v_f64),
                     "speedup_of_mixed_over_f64": (per_other / per_main) if other == "f64" else (per_main / per_other),
                     "lsqr_fp64_fallback": st2["lsqr_fp64_fallback"]}

    kern_f64 = kern if a.form == "f64" else kern_other
    kern_mixed = kern_other if a.form == "f64" else kern

    def sketch_rate(k, name, peak, issued_factor=None):
        rec = k.get(name)
        if not rec or rec["seconds"] <= 0:
            return None
        alg = 2.0 * s_rows * nnz * rec["launches"] / rec["seconds"] / 1e12
        out = {"kernel": name, "launches": rec["launches"], "s_per_launch": rec["seconds"] / rec["launches"],
               "tflops_algorithmic": alg, "frac_of_peak": alg / peak, "peak_tflops": peak,
               "flops_per_launch": 2.0 * s_rows * nnz}
        if issued_factor:
            out["tflops_matrix_core_issued"] = alg * issued_factor
            out["issued_over_algorithmic"] = issued_factor
        return out

    lowp_name = {"bf16": "sketch_bf16", "fp8": "sketch_fp8"}[a.sketch_prec]
    lowp_peak = PEAK_BF16_TFLOPS if a.sketch_prec == "bf16" else PEAK_FP8_TFLOPS
    issued = None
    if kern_mixed.get(lowp_name):
        nslots = sum(lp.sketch_operand_slots(b) for b in range(prob.nbox * prob.ncomp))
        pieces = 6 if a.sketch_prec == "bf16" else 12
        issued = nslots * 32.0 * prob.J * pieces / nnz
    sketch = {"f64": sketch_rate(kern_f64, "sketch_count" if a.sketch_kind == "count" else "sketch_f64",
                                 PEAK_FP64_TFLOPS),
              "mixed": sketch_rate(kern_mixed, lowp_name, lowp_peak, issued)}

    # HBM bandwidth this GPU reaches on a plain copy (read + write of 2 GiB each, 5 timed repetitions): the
    # measured ceiling the bandwidth-bound kernels are also compared with
    copy_b = 2 << 30
    src = torch.empty(copy_b // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2.0 * copy_b / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst

    def spmv(k, name, bj):
        rec = k.get(name)
        if not rec or rec["seconds"] <= 0:
            return None
        gbs = rec["bytes"] / rec["seconds"] / 1e9
        tb = TRAFFIC_BYTES.get(name) if a.workload == "gray-scott" else None
        return {"GB_s": gbs, "frac_of_hbm_peak": gbs / PEAK_HBM_GBS, "frac_of_measured_copy": gbs / copy_gbs,
                "launches": rec["launches"],
                "us_per_launch": 1e6 * rec["seconds"] / rec["launches"], "bytes_per_launch": rec["bytes"] / rec["launches"],
                "alg_bytes_formula": (f"nnz*{bj} + vectors (m+n)*8 (+ m*8 for the fused LSQR update)" if name != "trsv"
                                      else "n(n+1)/2*8 + vectors"),
                "traffic_bytes_per_launch": tb}

    lsqr_spmv = {"jmul_f64": spmv(kern_f64, "jmul", 8), "jtmul_f64": spmv(kern_f64, "jtmul", 8),
                 "jmul_f32": spmv(kern_mixed, "jmul_f32", 4), "jtmul_f32": spmv(kern_mixed, "jtmul_f32", 4),
                 "trsv": spmv(kern, "trsv", 8)}

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

    dtype = "f64" if a.form == "f64" else \
        f"f64 QR/TRSV/residual; {a.sketch_prec} sketch; {a.lsqr_prec} LSQR operator"
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
        "config": {"workload": workload, "n": n, "m": m, "s": s_rows, "nnz_J": nnz, "method": a.method,
                   "form": a.form,
                   "sketch": ("count_sketch_philox4x64_f64" if a.sketch_kind == "count" else
                              "gaussian_philox4x64_f64") if a.form == "f64" else
                             f"philox4x64_code_table_{a.sketch_prec}_exact_pieces",
                   "lsqr_tol": 1e-10, "outer_tol": 1e-10, "row_scale_c": 100.0, "initial_guess": "zero"},
        "relL2": rel,
        "relL2_target_met": bool(max(rel) <= 1e-6),
        "relL2_note": ("relL2 <= 1e-6 is out of reach on this workload for any solver: no coefficient vector of "
                       "its features fits u*, v* below 6.3e-6, 1.3e-5 on the test points "
                       "(tests/test_oracle_floor.py); the collocation solve's floor is 1.5e-4, 1.8e-4"
                       if a.workload == "gray-scott" else None),
        "newton": {"outer_iters": stats["outer_iters"], "jac_evals": stats["jac_evals"],
                   "lsqr_iters": stats["lsqr_iters"], "final_resnorm": stats["final_resnorm"],
                   "status": stats["status"], "lsqr_fp64_fallback": stats["lsqr_fp64_fallback"]},
        "mixed_form" if other == "mixed" else "f64_form": other_out,
        "sketch_tflops": sketch[a.form]["tflops_algorithmic"] if sketch[a.form] else None,
        "sketch": sketch,
        "lsqr_spmv_gbs": {k: (v["GB_s"] if v else None) for k, v in lsqr_spmv.items()},
        "lsqr_spmv": lsqr_spmv,
        "hbm_copy_GB_s": copy_gbs,
        "roofline": roof,
        "kernels": kernels,
    }
    lp.close()
    if not a.no_warm_start_study:
        # learned initial guess on a small member family of the same system (the full-size family would need
        # hundreds of full-size training solves): Newton steps and time against the zero guess on held-out
        # members, the FP64 solver deciding the answer
        from paper_2510_04170_amd import warmstart as WS
        print(f"[bench] warm-start study ({a.warm_train} training, {a.warm_test} held-out draws) ...",
              file=sys.stderr, flush=True)
        ws = WS.run(n_train=a.warm_train, n_test=a.warm_test)
        out["warm_start"] = {"family": ws["family"], "network": ws["network"], "seconds": ws["seconds"],
                             "mean": ws["mean"],
                             "max_field_diff_vs_zero_guess": max(r["field_diff"] for r in ws["per_draw"]),
                             "kept_fraction": float(np.mean([r["warm"]["kept"] for r in ws["per_draw"]])),
                             "fewer_jacobians_fraction": float(np.mean([r["warm"]["NJ"] < r["zero"]["NJ"]
                                                                        for r in ws["per_draw"]]))}
    if rank == 0 and not a.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.quick_cpu_baseline)
    if rank == 0:
        print(json.dumps(out), flush=True)
    del u
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
