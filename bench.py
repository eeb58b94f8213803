"""Benchmark: accelerated RPCholesky on one MI355X.

One step = one complete factorization (every round of proposals, residual
submatrix, rejection sampling, update GEMM, triangular solve and diagonal
update) of the mixture workload: N = 1e6 points in R^8 from a 10-component
Gaussian mixture, Gaussian kernel sigma = 2, k = 2000, b = 200.  Points are
resident in HBM before the timed region; F, pivots and workspace are
allocated once.

Prints one JSON line: pivots/s over the timed steps, the roofline of the
dominant kernel (the one-kernel round product of the BF16 modes, else the
update GEMM) from HIP-event timings taken inside the timed region, the
trace error against an FP64 run of the same problem, and the CPU oracle
timed on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_03969_amd import workloads as W  # noqa: E402

PEAKS = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "fp64_tflops": 78.6, "fp32_tflops": 157.3, "bf16_tflops": 2500.0,
}
PREC_BY_NAME = {v: k for k, v in W.PREC_NAMES.items()}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16", choices=sorted(PREC_BY_NAME))
    ap.add_argument("--workload", default="mixture", choices=["mixture", "laplace", "small", "sparse_hd"])
    ap.add_argument("--method", default="accel", choices=sorted(W.METHOD_NAMES.values()),
                    help="pivot rule: accel (Alg. 2, the method) or block (Alg. 7, a baseline)")
    ap.add_argument("--krr", action="store_true",
                    help="time kernel ridge regression by PCG (Section 3.2) with the preconditioner from arpc_factor")
    ap.add_argument("--qr", action="store_true",
                    help="time accelerated randomly pivoted QR (Alg. 5, FP64) on a synthetic 1000 x 100000 matrix")
    ap.add_argument("--lowmem", action="store_true",
                    help="time the low-memory implementation (Alg. 3, FP64) instead of arpc_factor")
    ap.add_argument("--b", type=int, default=0,
                    help="block size instead of the workload's (1 with --method accel: simple RPCholesky)")
    ap.add_argument("--cpu-rounds", type=int, default=3,
                    help="rounds of the oracle timed for the CPU baseline (0 = skip)")
    ap.add_argument("--no-compare-fp64", action="store_true",
                    help="skip the FP64 factorization that the trace-error ratio of a "
                         "reduced-precision mode is stated against")
    ap.add_argument("--serving", action="store_true",
                    help="run the serving stream instead (prints its own JSON line)")
    ap.add_argument("--serving-jobs", type=int, default=512)
    ap.add_argument("--serving-prec", default="bf16", choices=sorted(PREC_BY_NAME))
    ap.add_argument("--no-serving", action="store_true",
                    help="leave the serving stream out of the default run (it is measured after the "
                         "factorization and reported under 'serving')")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed region, copy a device buffer of this many MiB "
                         "once (a reference kernel for hardware byte counters)")
    return ap.parse_args()


KERNEL_SOURCES = {  # dominant kernel -> source file whose hash keys its counter summary
    "k_fused_round": "paper_2410_03969_amd/csrc/fused_kernels.hip",
    "k_panel": "paper_2410_03969_amd/csrc/mfma_kernels.hip",
}


def source_hash(rel: str) -> str:
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, dtype: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes, scaled by the copy-kernel
    factors recorded there), or None when no summary matches this workload or
    the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{dtype}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-record:"):
                for kv in line.split(":", 1)[1].split():
                    k, _, v = kv.partition("=")
                    fields[k] = v
    if fields.get("source_sha256_16") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    try:
        return float(fields["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def gemm_roofline(stats, prec, workload):
    """Roofline of the dominant kernel from the HIP-event kernel times: the
    one-kernel round product (BF16 modes) or the update-GEMM kernel.

    Algorithmic bytes per launch: F read over its k_r columns at the
    contraction precision, the points read, G written once to F at its
    storage precision, the row norms written (the two-kernel GEMM writes C
    instead).  The write of G into the panel-blocked copy that later rounds
    contract over is reported apart (blocked_copy_bytes_per_launch), as is
    the fraction with it counted.  Algorithmic flops: 2 N k_r s_r for the
    GEMM, plus N s_r^2 for the solve when fused, counted once although the
    three-product mode issues three BF16 products.  The binding roof (larger
    fraction) is reported first; the MFMA side also states the attainable
    fraction at the measured arithmetic intensity, min(1, AI * HBM / peak)."""
    ms = stats["ms_kernel"]["colgemm"]
    n = stats["launches"]["colgemm"]
    if ms <= 0 or n == 0:
        return None, None
    fused = bool(stats.get("fused"))
    kernel = "k_fused_round" if fused else "k_panel"
    sec = ms * 1e-3
    flops = stats["flops_colgemm"] + (stats["flops_trsm"] if fused else 0.0)
    tflops = flops / sec / 1e12
    gbs = stats["bytes_colgemm"] / sec / 1e9
    peak = {W.FP64: PEAKS["fp64_tflops"], W.FP32: PEAKS["fp32_tflops"]}.get(prec, PEAKS["bf16_tflops"])
    traffic = measured_traffic(kernel, workload, W.PREC_NAMES[prec])
    blocked = stats["bytes_blocked"] if fused else 0.0
    ai = flops / stats["bytes_colgemm"]
    attainable = min(peak, ai * PEAKS["hbm_gbs"] / 1e3)   # TFLOP/s at this intensity
    common = {"kernel": kernel, "avg_launch_ms": round(ms / n, 4), "launches": n,
              "algorithmic_bytes_per_launch": round(stats["bytes_colgemm"] / n),
              "blocked_copy_bytes_per_launch": round(blocked / n),
              "algorithmic_flops_per_launch": round(flops / n)}
    mf = {"bound": "mfma", "achieved": round(tflops, 3), "peak": peak, "unit": "TFLOP/s",
          "frac": round(tflops / peak, 4), "traffic": traffic,
          "intensity_flop_per_byte": round(ai, 1), "attainable": round(attainable, 1),
          "frac_of_attainable": round(tflops / attainable, 4), **common}
    hb = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
          "frac": round(gbs / PEAKS["hbm_gbs"], 4), "traffic": traffic,
          "frac_with_blocked_copy": round((stats["bytes_colgemm"] + blocked) / sec / 1e9 / PEAKS["hbm_gbs"], 4),
          **common}
    return (mf, hb) if mf["frac"] >= hb["frac"] else (hb, mf)


def cpu_baseline(X, prob, rounds, gpu_rounds):
    """The FP64 oracle (Alg. 2 with Alg. 1 in numpy) timed on this host on the
    first rounds of the same workload, and the full factorization's rate
    extrapolated from them (marked as such).

    Two timed samples: round 1 alone (k_r = 0: kernel columns, solve and
    diagonal only, cost beta N s per round) and rounds 1..R.  Their
    difference fixes alpha in the update-GEMM term alpha * 2 N k_r s_r, whose
    sum over a run is N (k^2 - sum_r s_r^2).  The full run's cost is then
    beta N k + alpha N (k^2 - sum s_r^2), with the GPU run's round count and
    equal rounds for sum s_r^2."""
    from oracle import PointsAccess, philox_stream, rpc_accel
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    blas_threads = None
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            blas_threads = max(int(i.get("num_threads", 1)) for i in info)
    except Exception:
        pass
    if blas_threads is None:
        blas_threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    t = time.perf_counter()
    r1 = rpc_accel(acc, prob.k, prob.b, philox_stream(prob.seed), max_rounds=1)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    rr = rpc_accel(acc, prob.k, prob.b, philox_stream(prob.seed), max_rounds=rounds)
    tr = time.perf_counter() - t
    N, k = prob.N, prob.k
    sizes = [int(v) for v in rr.round_sizes]
    beta = t1 / (N * max(sizes[0], 1))
    gemm_units, kr = 0.0, 0
    for s_ in sizes:
        gemm_units += 2.0 * N * kr * s_
        kr += s_
    rest = tr - beta * N * sum(sizes)
    alpha = max(rest, 0.0) / gemm_units if gemm_units > 0 else 0.0
    s_mean = k / max(gpu_rounds, 1)
    full_s = beta * N * k + alpha * N * (k * k - gpu_rounds * s_mean * s_mean)
    return {"value": round(k / full_s, 3), "unit": "pivots/s", "cores": int(cores),
            "blas_threads": int(blas_threads), "kind": "oracle", "extrapolated": True,
            "sample": f"rounds 1..{rounds} of the same workload ({rr.k_out} pivots in {tr:.1f} s, "
                      f"{rr.k_out / tr:.2f} pivots/s) and round 1 alone ({t1:.1f} s); full run "
                      f"extrapolated to {full_s:.0f} s with beta N k + alpha N (k^2 - sum s_r^2), "
                      f"{gpu_rounds} rounds",
            "sample_value": round(rr.k_out / tr, 3), "extrapolated_seconds": round(full_s, 1)}


def run_serving(args):
    print(json.dumps(serving_measure(args)), flush=True)


def serving_measure(args):
    """Serving stream: jobs shaped as in workloads.serving_stream (N log-uniform
    on [1e4, 2e5], d in {3, 8, 32}, k uniform on [200, 1500], b = k/10).  A
    closed loop with a bounded number of outstanding jobs measures the
    saturation throughput X_sat; then an open loop submits the same jobs at
    Poisson arrival times with rate 0.7 X_sat and reports the p50/p99 latency
    (submission to completion, timed by the library), the aggregate pivots/s
    and the mean number of resident jobs."""
    import torch
    from paper_2410_03969_amd import binding as B
    B.lib()
    prec = PREC_BY_NAME[args.serving_prec]
    jobs = W.serving_stream(n_jobs=args.serving_jobs, rate=1.0, prec=prec)
    dev = torch.device("cuda:0")
    Xs = [torch.from_numpy(j.X).to(dev) for j in jobs]
    torch.cuda.synchronize()
    budget = int(args.serving_budget_gb * (1 << 30))

    def run(arrivals, max_outstanding):
        srv = B.Server(budget, max_slots=args.serving_slots)
        lat, pivots, resident = [], 0, []
        pending = {}
        i = 0
        t0 = time.perf_counter()
        try:
            while i < len(jobs) or pending:
                now = time.perf_counter() - t0
                while (i < len(jobs) and len(pending) < max_outstanding
                       and (arrivals is None or arrivals[i] <= now)):
                    pending[srv.submit(Xs[i], jobs[i].problem)] = i
                    i += 1
                for h in list(pending):
                    r = srv.poll(h)
                    if r is not None:
                        del pending[h]
                        if r["status"] < 0:
                            raise RuntimeError(B.arpc_status_str(r["status"]))
                        lat.append(r["stats"]["ms_total"])
                        pivots += r["stats"]["k_out"]
                resident.append(srv.info()["active"])
                time.sleep(0.0002)
            span = time.perf_counter() - t0
            info = srv.info()
        finally:
            srv.close()
        return np.array(lat), pivots, span, float(np.mean(resident)), info

    lat_c, piv_c, span_c, res_c, _ = run(None, args.serving_slots * 4)
    x_sat = len(jobs) / span_c
    lam = 0.7 * x_sat
    arrivals = np.array([j.arrival for j in jobs]) / lam
    lat, piv, span, res, info = run(arrivals, len(jobs))
    out = {
        "metric": "serving latency", "unit": "ms", "n_gpus": 1, "dtype": W.PREC_NAMES[prec],
        "data": "synthetic", "higher_is_better": False,
        "config": {"workload": f"serving stream: {len(jobs)} jobs, N log-uniform [1e4, 2e5], "
                               f"d in {{3, 8, 32}}, k uniform [200, 1500], b = k/10, Gaussian sigma = sqrt(d)",
                   "slots": args.serving_slots, "budget_gb": args.serving_budget_gb},
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "arrival_rate_jobs_per_s": round(lam, 3), "saturation_jobs_per_s": round(x_sat, 3),
        "pivots_per_s": round(piv / span, 1), "mean_resident_jobs": round(res, 3),
        "mean_pivots_per_job": round(piv / len(jobs), 1),
        "peak_active": info["peak_active"], "peak_bytes": info["peak_bytes"],
        "ticks": info["ticks"], "ticked_jobs": info["ticked_jobs"],
        "closed_loop": {"pivots_per_s": round(piv_c / span_c, 1), "mean_resident_jobs": round(res_c, 3),
                        "p50_ms": round(float(np.percentile(lat_c, 50)), 3)},
    }
    del Xs
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.serving:
        return run_serving(args)
    import torch

    from paper_2410_03969_amd import binding as B

    B.lib()
    if args.qr:
        return run_qr(args, B, torch)
    if args.krr:
        return run_krr(args, B, torch)
    gen = {"mixture": W.mixture, "laplace": W.laplace, "small": W.small,
           "sparse_hd": W.sparse_hd}[args.workload]
    X, prob = gen()
    prec = PREC_BY_NAME[args.prec]
    prob = prob.with_(prec=prec)
    method = {v: k for k, v in W.METHOD_NAMES.items()}[args.method]
    variant = args.workload
    if args.b > 0 or method != W.ACCEL:
        prob = prob.with_(b=args.b if args.b > 0 else prob.b, method=method)
        variant = f"{args.workload}_{args.method}_b{prob.b}"   # no counter record for a variant
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    if args.lowmem:
        return run_lowmem(args, B, torch, X, Xd, prob.with_(prec=W.FP64), variant)
    pr = B.make_problem(prob)
    fdt = torch.float64 if prec == W.FP64 else torch.float32
    Ft = torch.empty((prob.k, prob.N), dtype=fdt, device=dev)
    piv = torch.empty(prob.k, dtype=torch.int64, device=dev)
    nbytes = B.arpc_workspace_size(pr)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step(classes):
        B.arpc_set_profiling_classes(classes)
        st, stats = B.arpc_factor(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(),
                                  nbytes, stream.cuda_stream)
        if st < 0:
            raise RuntimeError(B.arpc_status_str(st))
        return stats.as_dict()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step([])
    torch.cuda.synchronize()
    # the timed steps carry HIP events around the round-product kernels only
    # (the roofline's kernel); the per-class breakdown comes from one more,
    # untimed step with every class timed
    t0 = time.perf_counter()
    runs = [step(["colgemm", "trsm"]) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    breakdown = step(list(B.KERNEL_CLASSES))
    torch.cuda.synchronize()
    B.arpc_set_profiling(False)

    k_out = sum(r["k_out"] for r in runs)
    last = runs[-1]
    F = Ft[: last["k_out"]]
    normF2 = float((F.double() ** 2).sum().item())
    trace_err = (last["trace_A"] - normF2) / last["trace_A"]
    # roofline over all timed steps
    agg = dict(last)
    agg["fused"] = last.get("fused", 0)
    agg["ms_kernel"] = {c: sum(r["ms_kernel"][c] for r in runs) for c in B.KERNEL_CLASSES}
    agg["launches"] = {c: sum(r["launches"][c] for r in runs) for c in B.KERNEL_CLASSES}
    for key in ("flops_colgemm", "bytes_colgemm", "flops_trsm", "bytes_trsm", "bytes_blocked"):
        agg[key] = sum(r[key] for r in runs)
    roof, roof_alt = gemm_roofline(agg, prec, variant)

    out = {
        "metric": "pivots/s", "value": round(k_out / elapsed, 2), "unit": "pivots/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": W.PREC_NAMES[prec], "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={prob.N} d={prob.d} "
                               f"{W.KERNEL_NAMES[prob.kernel]} sigma={prob.sigma} "
                               f"k={prob.k} b={prob.b}"
                               + ("" if method == W.ACCEL else f" method={args.method}"),
                   "N": prob.N, "d": prob.d, "k": prob.k, "b": prob.b, "method": args.method,
                   "parallelism": "single GPU"},
        "roofline": roof, "roofline_alt": roof_alt,
        "rounds": last["rounds"], "acceptance": round(last["k_out"] / last["proposals"], 4),
        "trace_error_F": trace_err,
        "kernel_ms_per_step": {c: round(v, 3) for c, v in breakdown["ms_kernel"].items()},
    }
    if not args.no_compare_fp64 and prec != W.FP64:
        p64 = prob.with_(prec=W.FP64)
        out64 = B.factor(Xd, p64)
        F64 = out64["F"][:, : out64["stats"]["k_out"]]
        te64 = (out64["stats"]["trace_A"] - float((F64 ** 2).sum().item())) / out64["stats"]["trace_A"]
        out["fp64_compare"] = {"ms": round(out64["stats"]["ms_total"], 2), "trace_error_F": te64,
                               "ratio": trace_err / te64 if te64 > 0 else None}
        del out64, F64
    if not args.no_serving and args.workload == "mixture" and method == W.ACCEL:
        del F, Ft, piv, ws
        torch.cuda.empty_cache()
        srv = serving_measure(args)
        out["serving"] = {k: srv[k] for k in ("p50_ms", "p99_ms", "saturation_jobs_per_s",
                                             "arrival_rate_jobs_per_s", "pivots_per_s", "mean_pivots_per_job",
                                             "mean_resident_jobs", "dtype", "closed_loop", "peak_active",
                                             "ticks", "ticked_jobs")}
        out["serving"]["workload"] = srv["config"]["workload"]
    if args.cpu_rounds > 0 and method == W.ACCEL:
        out["cpu_baseline"] = cpu_baseline(X, prob, args.cpu_rounds, last["rounds"])
    print(json.dumps(out), flush=True)


def run_krr(args, B, torch):
    """Kernel ridge regression as in Section 3.2 on synthetic data: N = 20000
    points uniform on [0,1]^8, Matern-5/2 with bandwidth sqrt(d), mu = 1e-9 N,
    y = sum_j sin(3 x_j) + 0.01 noise; preconditioner from arpc_factor (FP64,
    k = 1000, b = 100); PCG to |r| <= 1e-8 |y|.  Plain CG (k = 0) runs for at
    most five times the preconditioned iteration count."""
    N, d, k, b = 20_000, 8, 1000, 100
    rng = np.random.default_rng(0)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.01 * rng.standard_normal(N)
    sigma, mu = float(np.sqrt(d)), 1e-9 * N
    prob = W.Problem(N=N, d=d, k=k, b=b, kernel=W.MATERN52, sigma=sigma, seed=0, prec=W.FP64)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    yd = torch.from_numpy(y).to(dev)
    for _ in range(args.warmup):
        fac = B.factor(Xd, prob)
        B.krr_pcg(Xd, yd, fac["F"], W.MATERN52, sigma, mu, tol=1e-8, max_iter=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = B.factor(Xd, prob)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = B.krr_pcg(Xd, yd, fac["F"], W.MATERN52, sigma, mu, tol=1e-8, max_iter=2000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    it = out["stats"]["iterations"]
    plain = B.krr_pcg(Xd, yd, None, W.MATERN52, sigma, mu, tol=1e-8, max_iter=5 * it)
    res = {
        "metric": "seconds to solve", "value": round(t2 - t0, 4), "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": round(1e3 * (t2 - t0), 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"krr: N={N} d={d} matern52 sigma=sqrt(d) mu=1e-9 N k={k} b={b} tol=1e-8",
                   "N": N, "d": d, "k": k, "b": b, "parallelism": "single GPU"},
        "roofline": None,
        "factor_ms": round(1e3 * (t1 - t0), 2), "pcg_ms": round(1e3 * (t2 - t1), 2), "pcg_iterations": it,
        "pcg_stats": out["stats"],
        "plain_cg": {"iterations": plain["stats"]["iterations"], "rel_residual": plain["stats"]["rel_residual"],
                     "converged": plain["status"] == 0, "ms": round(plain["stats"]["ms_total"], 2)},
    }
    print(json.dumps(res), flush=True)


def run_qr(args, B, torch):
    """Pivots/s of accelerated randomly pivoted QR on a seeded low-rank-plus-
    noise matrix (M = 1000, N = 100000, k = 500, b = 100), FP64."""
    M, N, k, b = 1000, 100_000, 500, 100
    Bm = W.qr_matrix(M, N)
    dev = torch.device("cuda:0")
    Bd = torch.from_numpy(np.ascontiguousarray(Bm.T)).to(dev).t()   # M x N view, column-major storage
    for _ in range(args.warmup):
        B.qr_factor(Bd, k, b, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [B.qr_factor(Bd, k, b, seed=0) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.arpc_set_profiling(True)
    breakdown = B.qr_factor(Bd, k, b, seed=0)["stats"]
    B.arpc_set_profiling(False)
    last = runs[-1]["stats"]
    out = {
        "metric": "pivots/s", "value": round(sum(r["stats"]["k_out"] for r in runs) / elapsed, 2),
        "unit": "pivots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"qr: M={M} N={N} rank 300 decay 0.99 noise 1e-5 k={k} b={b} (Alg. 5)",
                   "M": M, "N": N, "k": k, "b": b, "parallelism": "single GPU"},
        "roofline": None, "rounds": last["rounds"],
        "residual_rel_frobenius": float(np.sqrt(max(last["trace_resid"], 0.0) / last["trace_A"])),
        "kernel_ms_per_step": {c: round(v, 3) for c, v in breakdown["ms_kernel"].items()},
    }
    print(json.dumps(out), flush=True)


def run_lowmem(args, B, torch, X, Xd, prob, variant):
    """Pivots/s of the low-memory implementation (FP64), with its device
    footprint beside that of arpc_factor (workspace + F) on the same problem."""
    pr = B.make_problem(prob)
    dev = Xd.device
    Lt = torch.empty((prob.k, prob.k), dtype=torch.float64, device=dev)
    piv = torch.empty(prob.k, dtype=torch.int64, device=dev)
    nbytes = B.arpc_lowmem_workspace_size(pr)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step(classes):
        B.arpc_set_profiling_classes(classes)
        st, stats = B.arpc_factor_lowmem(pr, Xd.data_ptr(), Lt.data_ptr(), piv.data_ptr(), ws.data_ptr(), nbytes,
                                         stream.cuda_stream)
        if st < 0:
            raise RuntimeError(B.arpc_status_str(st))
        return stats.as_dict()

    for _ in range(args.warmup):
        step([])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step([]) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    breakdown = step(list(B.KERNEL_CLASSES))
    B.arpc_set_profiling(False)
    last = runs[-1]
    std_bytes = B.arpc_workspace_size(pr) + 8 * prob.N * prob.k
    out = {
        "metric": "pivots/s", "value": round(sum(r["k_out"] for r in runs) / elapsed, 2), "unit": "pivots/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{variant}: N={prob.N} d={prob.d} {W.KERNEL_NAMES[prob.kernel]} "
                               f"sigma={prob.sigma} k={prob.k} b={prob.b} low-memory (Alg. 3)",
                   "N": prob.N, "d": prob.d, "k": prob.k, "b": prob.b, "parallelism": "single GPU"},
        "roofline": None,
        "rounds": last["rounds"], "trace_error": (last["trace_resid"]) / last["trace_A"],
        "device_bytes": nbytes + 8 * prob.k * prob.k, "device_bytes_standard_fp64": std_bytes,
        "kernel_ms_per_step": {c: round(v, 3) for c, v in breakdown["ms_kernel"].items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
