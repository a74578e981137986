"""Benchmark: fine DOF/s per full multigrid eigensolve at 1e-8 relative lambda error.

One "step" is one complete FMG eigensolve (Algorithm 3.2 plus the tolerance loop on the
finest level) of the 2D Gross-Pitaevskii workload: unit square, W = x^2 + y^2, zeta = 100,
coarsest h = 1/16 refined 7 times to h = 1/2048 (4,190,209 fine DOF), m = 1, p = 2,
SGS(2,2) V-cycles, finest-level correction steps until |dlambda|/lambda <= 1e-9.  The
inputs are analytic (no data); the solver's working set is resident in HBM before timing.

Prints one JSON line.  value = fine DOF / mean seconds per solve (FP64 path); the mixed
path (FP32 V-cycles in FP64 refinement) is reported beside it, with p50/p99 latencies,
the error against the oracle's converged eigenvalue, the roofline of the dominant kernel
and the oracle timed on the host CPU on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "fine DOF/s per FMG eigensolve at 1e-8 λ err, mixed vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
TOL = 1e-9


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def time_solves(prob, opts, steps, warmup):
    import torch
    from paper_1502_04657_amd import Solver
    s = Solver(prob, opts)
    u = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        s.solve(u)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        res, _ = s.solve(u)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return res, u, total, lat


def smoother_roofline(prob, reps=20):
    """Average duration of the finest-level red-black half sweep (the V-cycle's dominant
    kernel) measured with HIP events on the stream it is launched on; algorithmic bytes
    per half sweep: read the other colour of x and f of this colour, write this colour
    of x = 1.5 * N * 8 bytes."""
    import torch
    from paper_1502_04657_amd import ops
    n, dim = prob.n_fine, prob.dim
    N = (n - 1) ** dim
    g = torch.Generator(device="cuda").manual_seed(0)
    x = ops.pack(dim, n, torch.randn(N, dtype=torch.float64, device="cuda", generator=g))
    f = ops.pack(dim, n, torch.randn(N, dtype=torch.float64, device="cuda", generator=g))
    ops.smooth(dim, n, x, f, 2)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ops.smooth(dim, n, x, f, 2)    # 5 half sweeps per call
    e1.record(st)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / (5 * reps)
    algo = 1.5 * N * 8
    achieved = algo / dt / 1e9
    return {"kernel": "k_smooth_half<2,double> (finest level)", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "avg_launch_us": dt * 1e6, "algorithmic_bytes_per_launch": algo}


def cpu_baseline():
    """The oracle, as it stands, on a bounded sample of the same workload family: the same
    problem (zeta = 100, W = x^2 + y^2, coarsest h = 1/16, same schedule and tolerance)
    refined 4 times (n = 256, 65,025 DOF) instead of 7."""
    from threadpoolctl import threadpool_limits

    from oracle import fmg as ofmg
    prob = W.Problem(2, 16, 4, (1.0, 1.0, 0.0), 0.0, 100.0)
    opts = W.Options(tol_lambda=TOL)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = ofmg.fmg(prob, opts)
        dt = time.perf_counter() - t0
    return {"value": prob.dofs() / dt, "unit": "fine DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FMG solve of the same workload at n=256 ({prob.dofs()} DOF, zeta=100, "
                      f"tol {TOL:g}), {dt:.1f} s single-threaded, lambda={r.lam:.12f}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; instances shard across GPUs with no communication "
              "(see the design notes), but no multi-GPU figure is produced. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = W.LARGE_2D
    N = prob.dofs()
    lam_ref = None
    gpath = os.path.join(ROOT, "tests", "golden", "large_2d.json")
    if os.path.exists(gpath):
        lam_ref = json.load(open(gpath))["large_2d"]["lambda_ref"]

    print(f"bench: FP64 {args.warmup}+{args.steps} solves, n={prob.n_fine}", file=sys.stderr, flush=True)
    res, u, total, lat = time_solves(prob, W.Options(tol_lambda=TOL), args.steps, args.warmup)
    ms = total / args.steps * 1e3
    out = {"metric": METRIC, "value": N / (total / args.steps), "unit": "fine DOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D GP ground state on [0,1]^2, W=x^2+y^2, zeta=100, P1 on right-triangle "
                                  "meshes, coarsest h=1/16 refined 7x to h=1/2048 (4,190,209 DOF), m=1 p=2 "
                                  "SGS(2,2) V-cycles, finest steps until |dlambda|/lambda<=1e-9",
                      "precision": "fp64", "global_batch": 1},
           "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
           "lambda": res.lam, "lambda_rq": res.lambda_rq, "steps_total": res.steps_total,
           "newton_total": res.newton_total, "factorizations": res.factor_total,
           "lambda_rel_err_vs_oracle": (abs(res.lam - lam_ref) / lam_ref) if lam_ref else None}
    if not args.no_mixed:
        print("bench: mixed precision", file=sys.stderr, flush=True)
        rm, _, tm, latm = time_solves(prob, W.Options(tol_lambda=TOL, precision="mixed"), args.steps, args.warmup)
        out["mixed"] = {"value": N / (tm / args.steps), "ms_per_step": tm / args.steps * 1e3,
                        "latency_ms": {"p50": _pct(latm, 50) * 1e3, "p99": _pct(latm, 99) * 1e3},
                        "lambda": rm.lam, "steps_total": rm.steps_total,
                        "lambda_rel_err_vs_oracle": (abs(rm.lam - lam_ref) / lam_ref) if lam_ref else None}
    print("bench: roofline", file=sys.stderr, flush=True)
    out["roofline"] = smoother_roofline(prob)
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
