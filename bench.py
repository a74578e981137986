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


VPOST_KERNEL = "k_vpost2d<double, 5, 54, 22, 256>"
PMC_FILE = os.path.join(ROOT, "profiles", "k_vpost2d_f64_pmc.md")
VPOST_SRC = os.path.join(ROOT, "paper_1502_04657_amd", "csrc", "vcycle2d.hip")


def _pmc_traffic():
    """HBM bytes per launch of the fused post pass from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on the finest-level
    unpack copy of known size), or None when the kernel source changed since."""
    import hashlib
    import re
    if not os.path.exists(PMC_FILE):
        return None
    txt = open(PMC_FILE).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    h = re.search(r"vcycle2d_sha256:\s*([0-9a-f]{64})", txt)
    if not m or not h:
        return None
    cur = hashlib.sha256(open(VPOST_SRC, "rb").read()).hexdigest()
    return float(m.group(1)) if cur == h.group(1) else None


def vpost_roofline(prob, steps):
    """Roofline of the fused FP64 post-smoothing level pass (prolongation-add + 5 red-black
    half sweeps; 54 x 22-tile build) on the finest level n = 2048, the largest HBM-bound
    kernel of the solve: start/stop HIP events stamped by each launch's own dispatch on its
    stream (hipExtLaunchKernel) for every finest-level launch during `steps` solves of the
    benchmark workload; algorithmic bytes per launch = 8 (3 N_l + N_{l-1}), N_l = 2047^2
    fine and N_{l-1} = 1023^2 coarse interior nodes."""
    import ctypes as C
    import torch
    from paper_1502_04657_amd import Solver, _ffi, lib
    s = Solver(prob, W.Options(tol_lambda=TOL))
    u = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    s.solve(u)
    torch.cuda.synchronize()
    L = lib()
    if L.fmg_profile_begin(_ffi.FMG_PROF_VPOST2D_F64, 16 * (steps + 1)) != 0:
        raise RuntimeError(L.fmg_last_error().decode())
    for _ in range(steps):
        s.solve(u)
    prof = _ffi.fmg_kernel_profile()
    if L.fmg_profile_end(C.byref(prof)) != 0:
        raise RuntimeError(L.fmg_last_error().decode())
    achieved = prof.bytes / prof.seconds / 1e9
    return {"kernel": VPOST_KERNEL, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": _pmc_traffic(),
            "avg_launch_us": prof.seconds / prof.launches * 1e6,
            "algorithmic_bytes_per_launch": prof.bytes / prof.launches, "launches": prof.launches}


def copy_calibration():
    """A plain copy of known size for scaling memory counters: the unpack of a cold padded
    n = 8192 level array (8191^2 interior doubles read, the same number written), after a
    1 GiB fill has pushed it out of the caches."""
    import torch
    from paper_1502_04657_amd import ops
    n = 8192
    N = (n - 1) ** 2
    lv = ops.new_level(2, n, device="cuda")
    lv.fill_(1.0)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    flush.fill_(2.0)
    torch.cuda.synchronize()
    out = ops.unpack(2, n, lv)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "k_unpack", "read_bytes": 8 * N, "write_bytes": 8 * N,
                                           "check": float(out[:4].sum().item())}}))


def bench_batch(steps, warmup, count=64):
    """Config 4: `count` uneven 2D instances (workloads.batch_instances, seed 0) per
    fmg_batch_solve call, mixed precision, tolerance 1e-9 on |dlambda|/lambda.  value =
    fine DOF of the batch / seconds per call; latency = each instance's completion time
    within its call.  The same instances solved one after another through fmg_solve are
    timed beside it."""
    import torch
    from paper_1502_04657_amd import Solver, batch_solve
    probs = W.batch_instances(count, 0)
    opts = W.Options(tol_lambda=TOL, precision="mixed")
    dofs = sum(p.dofs() for p in probs)
    for _ in range(warmup):
        batch_solve(probs, opts, check=False)
    torch.cuda.synchronize()
    lat, fails = [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = batch_solve(probs, opts, check=False)
        lat += [r.seconds for r in res]
        fails += sum(r.status != 0 for r in res)
    total = time.perf_counter() - t0
    solvers = [Solver(p, opts) for p in probs]
    for s in solvers:
        s.solve(check=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in solvers:
        s.solve(check=False)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    return {"metric": "fine DOF/s, batched FMG eigensolves (mixed precision, 1e-8 lambda)",
            "value": dofs * steps / total, "unit": "fine DOF/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": total / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": f"{count} 2D GP instances, n in {{256,512,1024}}, zeta log-uniform [0.1,1000], "
                                   "W=a x^2+b y^2, a,b in [0.5,2], coarsest h=1/16, seed 0", "global_batch": count},
            "instance_latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
            "failed_instances": fails, "sequential_fmg_solve_ms": seq * 1e3,
            "speedup_vs_sequential": seq / (total / steps)}


def bench_serve(count, budget_gb, rates=(0.5, 0.9, 1.25)):
    """Config 5: a request stream (workloads.serving_requests, seed 1) through one server.
    Saturation throughput = requests / time with all submitted at once; then Poisson
    arrivals (seed 2) at fractions of it.  Latency = submission to completion (device
    work observed done by the server), admission wait reported separately."""
    import torch
    from paper_1502_04657_amd import Server
    reqs = W.serving_requests(count, 1)
    opts = W.Options(tol_lambda=TOL, precision="mixed")
    budget = int(budget_gb * (1 << 30))

    def run(arrivals):
        out = {}
        with Server(hbm_budget=budget, max_slots=16) as sv:
            t0 = time.perf_counter()
            tickets, i = [], 0
            while len(out) < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and arrivals[i] <= now:
                    tickets.append(sv.submit(reqs[i], opts))
                    i += 1
                for t in tickets:
                    if t not in out:
                        r = sv.poll(t, want_u=False, check=False)
                        if r is not None:
                            out[t] = r[0]
                time.sleep(50e-6)
            span = time.perf_counter() - t0
        res = list(out.values())
        return span, res

    run([0.0] * min(8, len(reqs)) + [0.0] * (len(reqs) - min(8, len(reqs))))   # warm-up
    span, res = run([0.0] * len(reqs))
    sat = len(reqs) / span
    rows = [{"rate_frac": "saturation", "solves_per_s": sat,
             "latency_ms": {"p50": _pct([r.seconds for r in res], 50) * 1e3,
                            "p99": _pct([r.seconds for r in res], 99) * 1e3},
             "failed": sum(r.status != 0 for r in res)}]
    rng = np.random.default_rng(2)
    for f in rates:
        gaps = rng.exponential(1.0 / (f * sat), size=len(reqs))
        arr = np.cumsum(gaps) - gaps[0]
        span, res = run(list(arr))
        lat = [r.seconds for r in res]
        wait = [r.wait_seconds for r in res]
        rows.append({"rate_frac": f, "offered_per_s": f * sat, "solves_per_s": len(reqs) / span,
                     "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
                     "wait_ms": {"p50": _pct(wait, 50) * 1e3, "p99": _pct(wait, 99) * 1e3},
                     "failed": sum(r.status != 0 for r in res)})
    dofs = sum(p.dofs() for p in reqs)
    return {"metric": "serving: solves/s and p50/p99 latency vs offered rate (mixed precision, 1e-8 lambda)",
            "value": sat, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{count} requests: 70% 2D n=2^k k in 7..11, 30% 3D n in {{64,128,192}}, "
                                   "zeta log-uniform [0.1,1000], anisotropic harmonic W, seed 1",
                       "hbm_budget_gb": budget_gb, "fine_dof_total": dofs},
            "rates": rows}


def bench_omega(steps, warmup, lam_ref):
    """The fixed-iteration-count variant of the augmented solves (Section 3.3) against
    solving each augmented problem to convergence, on the default workload: correction
    steps, nonlinear iterations and time to reach |dlambda|/lambda <= 1e-9."""
    rows = []
    for k in (0, 1, 2, 3):
        res, _, total, lat = time_solves(W.LARGE_2D, W.Options(tol_lambda=TOL, newton_fixed_iters=k), steps, warmup)
        rows.append({"newton_fixed_iters": k or "converged", "ms_per_solve": total / steps * 1e3,
                     "steps_total": res.steps_total, "newton_total": res.newton_total, "status": res.status,
                     "lambda_rel_err_vs_oracle": abs(res.lam - lam_ref) / lam_ref if lam_ref else None})
    return {"metric": "fixed-iteration augmented solves vs converged ones (2D n=2048, zeta=100)", "rows": rows}


def bench_paper(steps, warmup):
    """The setting of the paper's Examples 4.1 (zeta = 1) and 4.2 (zeta = 100): 3D unit cube,
    W = x^2 + y^2 + z^2, coarsest h = 1/8 refined to h = 1/128, m = p = 1 with 3 + 3 CG
    smoothing steps, one FMG pass (fixed schedule).  Per mesh: DOF, time per solve and per
    DOF (the linear-complexity trend of Tables 1-2), lambda, and its distance to the
    converged discrete eigenvalue of the same mesh; the default smoother (SGS(2,2),
    m = 1, p = 2) beside it."""
    from paper_1502_04657_amd import Solver
    rows = []
    for zeta in (1.0, 100.0):
        for refine in range(1, 5):
            prob = W.Problem(3, 8, refine, (1.0, 1.0, 1.0), 0.0, zeta)
            conv, _ = Solver(prob, W.Options(tol_lambda=1e-13, max_final_steps=200)).solve(check=False)
            row = {"zeta": zeta, "n": 8 << refine, "dof": prob.dofs(), "lambda_converged": conv.lam}
            for tag, opts in (("cg_m1p1", W.Options(m=1, p=1, nu_pre=3, nu_post=3, smoother="cg")),
                              ("sgs_m1p2", W.Options())):
                res, _, total, _ = time_solves(prob, opts, steps, warmup)
                ms = total / steps * 1e3
                row[tag] = {"ms": ms, "us_per_kdof": ms * 1e6 / prob.dofs(), "lambda": res.lam,
                            "rel_dist_to_converged": abs(res.lam - conv.lam) / conv.lam, "status": res.status}
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return {"metric": "paper setting (Examples 4.1/4.2): time per solve and per DOF vs mesh", "rows": rows}


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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a cold plain copy of known size (memory-counter scaling)")
    ap.add_argument("--workload", choices=["fmg2d", "batch", "serve", "omega", "paper"], default="fmg2d",
                    help="fmg2d: the default line; batch / serve: the batched and serving workloads")
    ap.add_argument("--requests", type=int, default=60, help="serve: requests per rate")
    ap.add_argument("--budget-gb", type=float, default=32.0, help="serve: HBM budget of the server")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: independent instances shard across GPUs with no communication, "
              "and no multi-GPU figure is produced. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch":
        print(json.dumps(bench_batch(args.steps, args.warmup)))
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args.requests, args.budget_gb)))
        return
    prob = W.LARGE_2D
    N = prob.dofs()
    lam_ref = None
    gpath = os.path.join(ROOT, "tests", "golden", "large_2d.json")
    if os.path.exists(gpath):
        lam_ref = json.load(open(gpath))["large_2d"]["lambda_ref"]
    if args.workload == "paper":
        print(json.dumps(bench_paper(args.steps, args.warmup)))
        return
    if args.workload == "omega":
        print(json.dumps(bench_omega(args.steps, args.warmup, lam_ref)))
        return

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
    out["roofline"] = vpost_roofline(prob, args.steps)
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
