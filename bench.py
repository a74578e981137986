"""Benchmark: fine DOF/s per full multigrid eigensolve at 1e-8 relative lambda error, mixed
precision against FP64, with p50/p99 latency.

Default workload (fmg3d): one "step" is one complete FMG eigensolve (Algorithm 3.2 plus the
tolerance loop on the finest level) of the 3D Gross-Pitaevskii problem on the unit cube:
W = x^2 + y^2 + z^2, zeta = 10, P1 on Kuhn tetrahedra, coarsest h = 1/4 refined 6 times to
h = 1/256 (16,581,375 interior DOF), m = 1, p = 2, SGS(2,2) V-cycles, finest-level
correction steps until |dlambda|/lambda <= 1e-9.  The inputs are analytic (no data); the
solver's working set is resident in HBM before timing and each solve runs in full inside
the timed region.

Prints one JSON line: value = fine DOF / mean seconds per solve on the FP64 path; the mixed
path (FP32 V-cycles inside FP64 refinement) beside it, with latency percentiles, the
difference between the two results, the error of both paths against the oracle's converged
solution of the same problem at 128^3 (stored by tests/golden/make_golden.py), the
roofline of the dominant kernel (the fine-grid moment pass, FP64 VALU-bound), the HBM
rooflines of the fused V-cycle level passes and the oracle timed on the host CPU on a
bounded sample.  --workload fmg2d gives the 2D line (n = 2048, zeta = 100); batch, serve,
omega and paper the other workloads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "fine DOF/s per FMG eigensolve at 1e-8 λ err, mixed vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TOL = 1e-9
CSRC = os.path.join(ROOT, "paper_1502_04657_amd", "csrc")
GOLDEN = os.path.join(ROOT, "tests", "golden")

# Algorithmic FP64 flops per unit of work (an FMA counts 2):
# k_moments_raw<3>, per fine cell, exact integration by the whole-cell tables:
#   u~ Y^b (8 corners x 20 monomials FMA) 320, gradient sums (8 x 3 FMA) 48,
#   u~^2 Y^b (27 corner pairs: product + 10 FMA) 567, u~^3 Y^b and u~^4 from the power sums of
#   each tetrahedron's vertex values (corner powers 24, per tetrahedron 65, scaling 10) 424,
#   |grad u~|^2 (6 tetrahedra x 10) 60,
#   shift to coarse-local coordinates (45 + 15 + 3 FMA and 9 powers) 141, accumulation 39.
MOMENTS3D_FLOPS_PER_CELL = 320 + 48 + 567 + 424 + 60 + 141 + 39
# k_rhs3_rows, per interior node: sums and differences of the 7 opposite stencil pairs 14,
#   mass-moment sums m0, M1, M2 over them (1 + 7, 12 and 3 + 21 FMA) 84, position weights of
#   M_W 32, scales 4, the nonlinear term from the star's 14 outer vertices (powers and 3 FMA)
#   112, 36 edges (product, two adds, FMA; doubled at the end) 184 and 24 triangles (FMA) 48,
#   its polynomial in u_i 8, scale 2, combination 4.
RHS3D_FLOPS_PER_NODE = 14 + 84 + 32 + 4 + 112 + 184 + 48 + 8 + 2 + 4


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def _pcts(xs):
    a = np.asarray(xs) * 1e3
    return {f"p{q}": float(np.percentile(a, q)) for q in (10, 50, 90, 99)}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


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


def _sha(*names):
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(CSRC, n), "rb").read())
    return h.hexdigest()


def _pmc_traffic(summary, kernel, sources):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE scaled by the same counters on a plain copy of known size), or
    None when the summary is missing or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch\[" + re.escape(kernel) + r"\]:\s*([0-9.eE+]+)", txt)
    h = re.search(r"sources_sha256\[" + re.escape(kernel) + r"\]:\s*([0-9a-f]{64})", txt)
    if not m or not h or h.group(1) != _sha(*sources):
        return None
    return float(m.group(1))


def profile_kernel(prob, opts, kind, steps):
    """Run `steps` solves with per-launch start/stop events on one kernel (the library's
    measurement hook: events stamped by each launch's own dispatch on its stream, finest
    level only); returns launches, mean duration and the algorithmic bytes and units of work
    per launch."""
    import ctypes as C
    import torch
    from paper_1502_04657_amd import Solver, _ffi, lib
    s = Solver(prob, opts)
    u = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    s.solve(u)
    torch.cuda.synchronize()
    L = lib()
    if L.fmg_profile_begin(kind, 64 * (steps + 1)) != 0:
        raise RuntimeError(L.fmg_last_error().decode())
    for _ in range(steps):
        s.solve(u)
    prof = _ffi.fmg_kernel_profile()
    if L.fmg_profile_end(C.byref(prof)) != 0:
        raise RuntimeError(L.fmg_last_error().decode())
    if prof.launches == 0:
        raise RuntimeError(f"profile kind {kind} recorded no launch")
    n = prof.launches
    return {"launches": n, "avg_launch_us": prof.seconds / n * 1e6, "bytes_per_launch": prof.bytes / n,
            "units_per_launch": prof.units / n, "seconds": prof.seconds}


def hbm_roofline(kernel, p, summary, sources):
    achieved = p["bytes_per_launch"] / (p["avg_launch_us"] * 1e-6) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": _pmc_traffic(summary, kernel, sources),
            "avg_launch_us": p["avg_launch_us"], "algorithmic_bytes_per_launch": p["bytes_per_launch"],
            "launches": p["launches"]}


def alu_roofline(kernel, p, flops_per_unit, summary, sources):
    flops = flops_per_unit * p["units_per_launch"]
    achieved = flops / (p["avg_launch_us"] * 1e-6) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": _pmc_traffic(summary, kernel, sources), "avg_launch_us": p["avg_launch_us"],
            "algorithmic_flops_per_launch": flops, "flops_per_unit": flops_per_unit,
            "units_per_launch": p["units_per_launch"],
            "achieved_gbs": p["bytes_per_launch"] / (p["avg_launch_us"] * 1e-6) / 1e9,
            "algorithmic_bytes_per_launch": p["bytes_per_launch"], "launches": p["launches"]}


def _m_norm(prob, n, v):
    """sqrt(v^T M v) on the fine mesh, by the library's Rayleigh-quotient reduction."""
    from paper_1502_04657_amd import ops
    return math.sqrt(ops.forms(prob, n, ops.pack(prob.dim, n, v))[2])


def rel_m_diff(prob, got, want):
    """Relative M-norm distance after sign alignment."""
    import torch
    s = 1.0 if float(torch.dot(got, want)) >= 0 else -1.0
    n = prob.n_fine
    return _m_norm(prob, n, s * got - want) / _m_norm(prob, n, want)


def _unfold_sym3(n, v):
    """Node (i, j, k) takes the stored value of its sorted index triple (the golden keeps the
    nodes i <= j <= k of the axis-permutation-symmetric ground state)."""
    m = n - 1
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    keep = (i <= j) & (j <= k)
    table = np.full((m, m, m), np.nan)
    table[keep] = v
    srt = np.sort(np.stack([i, j, k], axis=-1), axis=-1)
    out = table[srt[..., 2], srt[..., 1], srt[..., 0]]
    assert not np.isnan(out).any()
    return out.ravel()


def oracle_check_3d():
    """Both paths on the same problem at 128^3 (2,048,383 DOF) against the oracle's
    converged discrete solution stored in tests/golden/mid_3d.npz: relative lambda error
    and relative M-norm eigenvector error after sign alignment, at the benchmark tolerance."""
    import torch
    from paper_1502_04657_amd import Solver
    path = os.path.join(GOLDEN, "mid_3d.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    meta = json.loads(str(z["meta"]))
    p = meta["problem"]
    prob = W.Problem(p["dim"], p["n_coarse"], p["n_refine"], tuple(p["w_quad"]), p["w_const"], p["zeta"],
                     tuple(p.get("diffusion", (1.0, 1.0, 1.0))))
    lam_ref = float(z["lambda_ref"])
    u_ref = z["u_ref"]
    if meta["folded_sym3"]:
        u_ref = _unfold_sym3(prob.n_fine, u_ref)
    u_ref = torch.from_numpy(u_ref).cuda()
    out = {"workload": f"same problem at n = {prob.n_fine} ({prob.dofs()} DOF), tol {TOL:g}", "lambda_ref": lam_ref}
    for prec in ("fp64", "mixed"):
        r, u = Solver(prob, W.Options(tol_lambda=TOL, precision=prec)).solve()
        out[prec] = {"lambda": r.lam, "lambda_rel_err": abs(r.lam - lam_ref) / lam_ref,
                     "u_rel_err_M": rel_m_diff(prob, u, u_ref), "status": r.status}
    return out


def bench_fmg3d(args):
    import torch
    prob = W.LARGE_3D
    N = prob.dofs()
    print(f"bench: FP64 {args.warmup}+{args.steps} solves, 3D n={prob.n_fine}", file=sys.stderr, flush=True)
    res, u64, total, lat = time_solves(prob, W.Options(tol_lambda=TOL), args.steps, args.warmup)
    out = {"metric": METRIC, "value": N / (total / args.steps), "unit": "fine DOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "3D GP ground state on [0,1]^3, W=x^2+y^2+z^2, zeta=10, P1 on Kuhn tetrahedra, "
                                  "coarsest h=1/4 refined 6x to h=1/256 (16,581,375 DOF), m=1 p=2 SGS(2,2) "
                                  "V-cycles, finest steps until |dlambda|/lambda<=1e-9",
                      "precision": "fp64", "global_batch": 1},
           "latency_ms": _pcts(lat), "lambda": res.lam, "lambda_rq": res.lambda_rq, "residual": res.residual,
           "gamma_est": res.gamma_est, "steps_total": res.steps_total, "newton_total": res.newton_total,
           "status": res.status}
    if not args.no_mixed:
        print("bench: mixed precision", file=sys.stderr, flush=True)
        rm, um, tm, latm = time_solves(prob, W.Options(tol_lambda=TOL, precision="mixed"), args.steps, args.warmup)
        out["mixed"] = {"value": N / (tm / args.steps), "ms_per_step": tm / args.steps * 1e3,
                        "speedup_vs_fp64": total / tm, "latency_ms": _pcts(latm), "lambda": rm.lam,
                        "steps_total": rm.steps_total, "status": rm.status,
                        "lambda_rel_diff_vs_fp64": abs(rm.lam - res.lam) / res.lam,
                        "u_rel_diff_vs_fp64_M": rel_m_diff(prob, um, u64)}
        del um
    del u64
    torch.cuda.empty_cache()
    if not args.no_oracle:
        print("bench: 128^3 against the stored oracle solution", file=sys.stderr, flush=True)
        out["oracle_check_128"] = oracle_check_3d()
    print("bench: per-kernel events", file=sys.stderr, flush=True)
    from paper_1502_04657_amd import _ffi
    opts = W.Options(tol_lambda=TOL)
    psteps = max(2, min(args.steps, 10))
    pm = profile_kernel(prob, opts, _ffi.FMG_PROF_MOMENTS3D, psteps)
    pr = profile_kernel(prob, opts, _ffi.FMG_PROF_RHS3D, psteps)
    ppre = profile_kernel(prob, opts, _ffi.FMG_PROF_VPRE3D_F64, psteps)
    ppost = profile_kernel(prob, opts, _ffi.FMG_PROF_VPOST3D_F64, psteps)
    summary = "fmg3d_n256_pmc.md"
    out["roofline"] = alu_roofline("k_moments_raw<3>", pm, MOMENTS3D_FLOPS_PER_CELL, summary,
                                   ("moments.hip", "moment_tables.h"))
    out["rhs_roofline"] = alu_roofline("k_rhs3_rows", pr, RHS3D_FLOPS_PER_NODE, summary, ("grid.hip", "tables.h"))
    out["vcycle_roofline"] = [hbm_roofline("k_vpass3d<double, 3, 0, 0, 26, 26, 512>", ppre, summary,
                                           ("vcycle3d.hip", "grid.hip")),
                              hbm_roofline("k_vpass3d<double, 3, 2, 0, 26, 26, 512>", ppost, summary,
                                           ("vcycle3d.hip", "grid.hip"))]
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_3d()
    return out


def vpost_roofline_2d(prob, steps):
    """Roofline of the fused FP64 post-smoothing level pass (prolongation-add + 5 red-black
    half sweeps; 54 x 22-tile build) on the finest 2D level n = 2048: algorithmic bytes per
    launch = 8 (3 N_l + N_{l-1}), N_l = 2047^2 fine and N_{l-1} = 1023^2 coarse interior nodes."""
    from paper_1502_04657_amd import _ffi
    p = profile_kernel(prob, W.Options(tol_lambda=TOL), _ffi.FMG_PROF_VPOST2D_F64, steps)
    return hbm_roofline("k_vpost2d<double, 5, 54, 22, 256>", p, "fmg2d_n2048_pmc.md", ("vcycle2d.hip",))


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
    """Config 4: `count` uneven 2D instances (workloads.batch_instances, seed 0), mixed
    precision, tolerance 1e-9 on |dlambda|/lambda.  value = fine DOF of the batch / seconds
    per replay of a batch plan (each instance's kernels captured once into HIP graphs and
    replayed on 16 streams, 2D tile choices from the autotuner); latency = each instance's
    completion time within its replay.
    The same instances through fmg_batch_solve (no graphs, 8 streams, eight enqueueing host
    threads) and one after another through fmg_solve are timed beside it."""
    import torch
    from paper_1502_04657_amd import BatchPlan, Solver, batch_solve, tuning
    probs = W.batch_instances(count, 0)
    opts = W.Options(tol_lambda=TOL, precision="mixed")
    dofs = sum(p.dofs() for p in probs)
    # the 2D tile choices, measured now on the largest level of the batch (no cache)
    t0 = time.perf_counter()
    choice = tuning.autotune(2, max(p.n_fine for p in probs), "mixed", cache=None)
    t_tune = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = BatchPlan(probs, opts)
    t_create = time.perf_counter() - t0
    for _ in range(warmup):
        plan.run(check=False)
    torch.cuda.synchronize()
    lat, fails = [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = plan.run(check=False)
        lat += [r.seconds for r in res]
        fails += sum(r.status != 0 for r in res)
    total = time.perf_counter() - t0
    plan.close()
    for _ in range(warmup):
        batch_solve(probs, opts, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch_solve(probs, opts, check=False)
    tb = (time.perf_counter() - t0) / steps
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
            "failed_instances": fails, "tuning": choice, "autotune_ms": t_tune * 1e3,
            "plan_create_ms": t_create * 1e3,
            "batch_solve_ms": tb * 1e3, "sequential_fmg_solve_ms": seq * 1e3,
            "speedup_vs_batch_solve": tb / (total / steps), "speedup_vs_sequential": seq / (total / steps)}


def bench_serve(count, budget_gb, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.25)):
    """Config 5: a request stream (workloads.serving_requests, seed 1) through one server,
    with the real HBM budget (90 % of the free device memory, or --budget-gb) at six offered
    rates, and with a 4 GB budget, so that admission binds, at two.  Per budget: saturation throughput =
    requests / time with all submitted at once; then Poisson arrivals (seed 2) at fractions
    of it.  Latency = submission to completion (device work observed done by the server),
    the admission wait (submission to start) reported separately; failed requests are
    listed with their problem."""
    import torch
    from paper_1502_04657_amd import Server
    reqs = W.serving_requests(count, 1)
    opts = W.Options(tol_lambda=TOL, precision="mixed")
    real = budget_gb if budget_gb else 0.9 * torch.cuda.mem_get_info()[0] / (1 << 30)

    def run(items, arrivals, budget):
        out = {}
        with Server(hbm_budget=int(budget * (1 << 30)), max_slots=16) as sv:
            t0 = time.perf_counter()
            pending, i, shown, last = {}, 0, 0, 0.0
            while len(out) < len(items):
                now = time.perf_counter() - t0
                while i < len(items) and arrivals[i] <= now:
                    pending[sv.submit(items[i], opts)] = i
                    i += 1
                for t in list(pending):
                    r = sv.poll(t, want_u=False, check=False)
                    if r is not None:
                        out[pending.pop(t)] = r[0]
                # progress every 50 completions, and at least every 30 s
                if len(out) >= shown + 50 or now - last >= 30.0:
                    shown, last = len(out) // 50 * 50, now
                    print(f"bench: serving {len(out)}/{len(items)} done at {now:.1f} s", file=sys.stderr, flush=True)
                time.sleep(50e-6)
            span = time.perf_counter() - t0
        return span, [out[k] for k in range(len(items))]

    def row(tag, span, res, offered=None):
        lat = [r.seconds for r in res]
        wait = [r.wait_seconds for r in res]
        d3 = [r.seconds for r, p in zip(res, reqs) if p.dim == 3]
        d2 = [r.seconds for r, p in zip(res, reqs) if p.dim == 2]
        fails = [{"request": k, "dim": p.dim, "n": p.n_fine, "n_coarse": p.n_coarse, "zeta": p.zeta,
                  "status": r.status} for k, (r, p) in enumerate(zip(res, reqs)) if r.status != 0]
        out = {"rate_frac": tag, "solves_per_s": len(res) / span,
               "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
               "latency_ms_2d": {"p50": _pct(d2, 50) * 1e3, "p99": _pct(d2, 99) * 1e3},
               "latency_ms_3d": {"p50": _pct(d3, 50) * 1e3, "p99": _pct(d3, 99) * 1e3},
               "wait_ms": {"p50": _pct(wait, 50) * 1e3, "p99": _pct(wait, 99) * 1e3},
               "failed": len(fails), "failed_requests": fails}
        if offered is not None:
            out["offered_per_s"] = offered
        return out

    run(reqs[:40], [0.0] * 40, real)   # warm-up
    budgets = []
    # the 4 GB budget (admission binds) at saturation and two rates
    for budget, fracs in ((real, rates), (4.0, (0.5, 1.0))):
        print(f"bench: serving, budget {budget:.1f} GB, saturation", file=sys.stderr, flush=True)
        span, res = run(reqs, [0.0] * len(reqs), budget)
        sat = len(reqs) / span
        rows = [row("saturation", span, res)]
        print("bench: row " + json.dumps(rows[-1]), file=sys.stderr, flush=True)
        rng = np.random.default_rng(2)
        for f in fracs:
            print(f"bench: serving, budget {budget:.1f} GB, rate {f}", file=sys.stderr, flush=True)
            gaps = rng.exponential(1.0 / (f * sat), size=len(reqs))
            arr = np.cumsum(gaps) - gaps[0]
            span, res = run(reqs, list(arr), budget)
            rows.append(row(f, span, res, f * sat))
            print("bench: row " + json.dumps(rows[-1]), file=sys.stderr, flush=True)
        budgets.append({"hbm_budget_gb": budget, "saturation_solves_per_s": sat, "rates": rows})
    dofs = sum(p.dofs() for p in reqs)
    return {"metric": "serving: solves/s and p50/p99 latency vs offered rate (mixed precision, 1e-8 lambda)",
            "value": budgets[0]["saturation_solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{count} requests: 70% 2D n=2^k k in 7..11, 30% 3D n in {{64,128,192}} "
                                   "(coarsest mesh by zeta, workloads.coarse_cells_3d), zeta log-uniform "
                                   "[0.1,1000], anisotropic harmonic W, seed 1; Poisson arrivals seed 2",
                       "fine_dof_total": dofs},
            "budgets": budgets}


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


def _oracle_timed(prob):
    from threadpoolctl import threadpool_limits

    from oracle import fmg as ofmg
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = ofmg.fmg(prob, W.Options(tol_lambda=TOL))
        dt = time.perf_counter() - t0
    return r, dt


def cpu_baseline_3d():
    """The oracle, as it stands, on a bounded sample of the same workload family: the same
    problem (3D, zeta = 10, W = x^2+y^2+z^2, coarsest h = 1/4, same schedule and tolerance)
    refined 3 times (n = 32, 29,791 DOF) instead of 6, single-threaded."""
    prob = W.Problem(3, 4, 3, (1.0, 1.0, 1.0), 0.0, 10.0)
    r, dt = _oracle_timed(prob)
    model, avail = host_cpu()
    return {"value": prob.dofs() / dt, "unit": "fine DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FMG solve of the same workload at n=32 ({prob.dofs()} DOF, zeta=10, tol {TOL:g}), "
                      f"{dt:.1f} s single-threaded, lambda={r.lam:.12f}",
            "host_cpu": model, "host_cpus_available": avail}


def cpu_baseline_2d():
    """The oracle on the 2D workload family: the same problem (zeta = 100, W = x^2 + y^2,
    coarsest h = 1/16, same schedule and tolerance) refined 4 times (n = 256, 65,025 DOF)."""
    prob = W.Problem(2, 16, 4, (1.0, 1.0, 0.0), 0.0, 100.0)
    r, dt = _oracle_timed(prob)
    model, avail = host_cpu()
    return {"value": prob.dofs() / dt, "unit": "fine DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FMG solve of the same workload at n=256 ({prob.dofs()} DOF, zeta=100, "
                      f"tol {TOL:g}), {dt:.1f} s single-threaded, lambda={r.lam:.12f}",
            "host_cpu": model, "host_cpus_available": avail}


def bench_fmg2d(args):
    prob = W.LARGE_2D
    N = prob.dofs()
    lam_ref = None
    gpath = os.path.join(GOLDEN, "large_2d.json")
    if os.path.exists(gpath):
        lam_ref = json.load(open(gpath))["large_2d"]["lambda_ref"]
    print(f"bench: FP64 {args.warmup}+{args.steps} solves, n={prob.n_fine}", file=sys.stderr, flush=True)
    res, u, total, lat = time_solves(prob, W.Options(tol_lambda=TOL), args.steps, args.warmup)
    out = {"metric": METRIC, "value": N / (total / args.steps), "unit": "fine DOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D GP ground state on [0,1]^2, W=x^2+y^2, zeta=100, P1 on right-triangle "
                                  "meshes, coarsest h=1/16 refined 7x to h=1/2048 (4,190,209 DOF), m=1 p=2 "
                                  "SGS(2,2) V-cycles, finest steps until |dlambda|/lambda<=1e-9",
                      "precision": "fp64", "global_batch": 1},
           "latency_ms": _pcts(lat), "lambda": res.lam, "lambda_rq": res.lambda_rq, "steps_total": res.steps_total,
           "newton_total": res.newton_total, "factorizations": res.factor_total,
           "lambda_rel_err_vs_oracle": (abs(res.lam - lam_ref) / lam_ref) if lam_ref else None}
    if not args.no_mixed:
        print("bench: mixed precision", file=sys.stderr, flush=True)
        rm, _, tm, latm = time_solves(prob, W.Options(tol_lambda=TOL, precision="mixed"), args.steps, args.warmup)
        out["mixed"] = {"value": N / (tm / args.steps), "ms_per_step": tm / args.steps * 1e3,
                        "latency_ms": _pcts(latm), "lambda": rm.lam, "steps_total": rm.steps_total,
                        "lambda_rel_err_vs_oracle": (abs(rm.lam - lam_ref) / lam_ref) if lam_ref else None}
    print("bench: roofline", file=sys.stderr, flush=True)
    out["roofline"] = vpost_roofline_2d(prob, max(2, min(args.steps, 10)))
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_2d()
    return out


# ---- rocprofv3 database summaries (the text committed under profiles/) ------------------
def short_name(name):
    """'void fmg::(anonymous namespace)::k_x<a, b>(args)' -> 'k_x<a, b>'."""
    name = re.sub(r"^void ", "", name).replace("(anonymous namespace)::", "").replace("fmg::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return name[:i]
    return name


def rocpd_stats(db, top=25):
    import collections
    import sqlite3
    c = sqlite3.connect(db)
    st = collections.defaultdict(list)
    big = collections.defaultdict(list)
    for name, t0, t1, gx, gy, gz, vgpr, lds in c.execute(
            "select name, start, end, grid_x, grid_y, grid_z, vgpr_count, lds_size from kernels"):
        k = short_name(name)
        st[k].append((t1 - t0) * 1e-3)
        big[k].append((gx * gy * gz, (t1 - t0) * 1e-3, vgpr, lds))
    tot = sum(sum(v) for v in st.values())
    print(f"total kernel time {tot / 1e3:.3f} ms over {sum(len(v) for v in st.values())} dispatches\n")
    print("| kernel | calls | total ms | avg us | max us | % |\n|---|---:|---:|---:|---:|---:|")
    for k, v in sorted(st.items(), key=lambda kv: -sum(kv[1]))[:top]:
        print(f"| `{k}` | {len(v)} | {sum(v) / 1e3:.3f} | {sum(v) / len(v):.2f} | {max(v):.2f} | "
              f"{100 * sum(v) / tot:.1f} |")
    print("\nLargest-grid dispatches (the finest level) of the measured kernels:\n")
    print("| kernel | grid (threads) | dispatches | avg us | min us | max us | VGPRs | LDS B |\n"
          "|---|---:|---:|---:|---:|---:|---:|---:|")
    for k in PMC_KERNELS:
        if k not in big:
            continue
        g = max(x[0] for x in big[k])
        d = [x for x in big[k] if x[0] == g]
        ts = [x[1] for x in d]
        print(f"| `{k}` | {g} | {len(d)} | {sum(ts) / len(ts):.2f} | {min(ts):.2f} | {max(ts):.2f} | {d[0][2]} | "
              f"{d[0][3]} |")


PMC_KERNELS = {"k_moments_raw<3>": ("moments.hip", "moment_tables.h"), "k_rhs3_rows": ("grid.hip", "tables.h"),
               "k_newton<3, true, true, true>": ("small.hip",),
               "k_vpass3d<double, 3, 0, 0, 26, 26, 512>": ("vcycle3d.hip", "grid.hip"),
               "k_vpass3d<double, 3, 2, 0, 26, 26, 512>": ("vcycle3d.hip", "grid.hip"),
               "k_vpass3d<double, 2, 0, 1, 28, 28, 512>": ("vcycle3d.hip", "grid.hip"),
               "k_vpre2d<double, 5, 50, 34, 256>": ("vcycle2d.hip",),
               "k_vpost2d<double, 5, 54, 22, 256>": ("vcycle2d.hip",), "k_moments_raw<2>": ("moments.hip",),
               "k_rhs<2>": ("grid.hip", "tables.h")}


def _pmc_by_kernel(db):
    """Per kernel: (largest grid, mean counter KiB over the dispatches with that grid, count)."""
    import collections
    import sqlite3
    c = sqlite3.connect(db)
    st = collections.defaultdict(list)
    for name, gs, val in c.execute("select kernel_name, grid_size, value from counters_collection"):
        st[short_name(name)].append((gs, val))
    out = {}
    for k, v in st.items():
        g = max(x[0] for x in v)
        vals = [x[1] for x in v if x[0] == g]
        out[k] = (g, sum(vals) / len(vals), len(vals))
    return out


def rocpd_pmc(fetch_db, write_db, copy_fetch_db, copy_write_db):
    """Finest-level HBM traffic of the 3D kernels: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch, dispatches of the largest grid) scaled by the same counters on the cold
    n = 8192 unpack of --copy-calibration (8 * 8191^2 bytes read and written)."""
    known = 8 * 8191 ** 2 / 1024.0
    cf = _pmc_by_kernel(copy_fetch_db)["k_unpack"][1]
    cw = _pmc_by_kernel(copy_write_db)["k_unpack"][1]
    sf, sw = known / cf, known / cw
    print(f"| counter | copy kernel KiB | known KiB | scale |\n|---|---:|---:|---:|\n"
          f"| FETCH_SIZE | {cf:.1f} | {known:.1f} | {sf:.4f} |\n| WRITE_SIZE | {cw:.1f} | {known:.1f} | {sw:.4f} |\n")
    f, w = _pmc_by_kernel(fetch_db), _pmc_by_kernel(write_db)
    print("| kernel | grid | dispatches | FETCH KiB | WRITE KiB | scaled read MB | scaled write MB |\n"
          "|---|---:|---:|---:|---:|---:|---:|")
    lines = []
    for k, src in PMC_KERNELS.items():
        if k not in f or k not in w:
            continue
        g, fk, nd = f[k]
        wk = w[k][1]
        rd, wr = fk * 1024 * sf, wk * 1024 * sw
        print(f"| `{k}` | {g} | {nd} | {fk:.1f} | {wk:.1f} | {rd / 1e6:.2f} | {wr / 1e6:.2f} |")
        lines.append(f"traffic_bytes_per_launch[{k}]: {rd + wr:.0f}")
        lines.append(f"sources_sha256[{k}]: {_sha(*src)}")
    print()
    print("\n".join(lines))


def rocpd_counters(db):
    """Per-dispatch means of every counter of a rocprofv3 --pmc database (one or more
    counters per pass), for the kernels of PMC_KERNELS and the 3D residual-restriction and
    form-u kernels, over each kernel's dispatches with its largest grid."""
    import collections
    import sqlite3
    c = sqlite3.connect(db)
    want = set(PMC_KERNELS) | {"k_resid_restrict<3, double>", "k_form_u<3>"}
    st = collections.defaultdict(lambda: collections.defaultdict(list))
    durs = collections.defaultdict(dict)
    for name, cn, gs, val, disp, dur in c.execute(
            "select kernel_name, counter_name, grid_size, value, dispatch_id, duration from counters_collection"):
        k = short_name(name)
        if k in want:
            st[k][cn].append((gs, val))
            durs[k][disp] = (gs, dur)
    names = sorted({cn for d in st.values() for cn in d})
    print("| kernel | grid | dispatches | duration us | " + " | ".join(names) + " |")
    print("|---|---:|---:|---:|" + "---:|" * len(names))
    for k in sorted(st):
        g = max(x[0] for v in st[k].values() for x in v)
        ds = [d for gs, d in durs[k].values() if gs == g]
        cells = []
        for cn in names:
            vals = [x[1] for x in st[k].get(cn, []) if x[0] == g]
            cells.append(f"{sum(vals) / len(vals):,.0f}" if vals else "")
        print(f"| `{k}` | {g} | {len(ds)} | {sum(ds) / len(ds) / 1e3:.1f} | " + " | ".join(cells) + " |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="fmg3d: skip the 128^3 check against the stored oracle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a cold plain copy of known size (memory-counter scaling)")
    ap.add_argument("--rocpd-stats", metavar="DB", help="print the kernel summary of a rocprofv3 database and exit")
    ap.add_argument("--rocpd-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print the scaled FETCH/WRITE traffic of the 3D kernels from four --pmc databases")
    ap.add_argument("--rocpd-counters", metavar="DB",
                    help="print per-kernel means of every counter of a rocprofv3 --pmc database")
    ap.add_argument("--workload", choices=["fmg3d", "fmg2d", "batch", "serve", "omega", "paper"], default="fmg3d",
                    help="fmg3d: the default line (3D 256^3); fmg2d: 2D n = 2048; batch / serve: the batched "
                         "and serving workloads")
    ap.add_argument("--requests", type=int, default=500, help="serve: requests per rate")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serve: HBM budget of the first pass (default: 90%% of free device memory)")
    args = ap.parse_args()
    if args.rocpd_stats:
        rocpd_stats(args.rocpd_stats)
        return
    if args.rocpd_pmc:
        rocpd_pmc(*args.rocpd_pmc)
        return
    if args.rocpd_counters:
        rocpd_counters(args.rocpd_counters)
        return
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
    elif args.workload == "serve":
        print(json.dumps(bench_serve(args.requests, args.budget_gb)))
    elif args.workload == "paper":
        print(json.dumps(bench_paper(args.steps, args.warmup)))
    elif args.workload == "omega":
        gpath = os.path.join(GOLDEN, "large_2d.json")
        lam_ref = json.load(open(gpath))["large_2d"]["lambda_ref"] if os.path.exists(gpath) else None
        print(json.dumps(bench_omega(args.steps, args.warmup, lam_ref)))
    elif args.workload == "fmg2d":
        print(json.dumps(bench_fmg2d(args)))
    else:
        print(json.dumps(bench_fmg3d(args)))


if __name__ == "__main__":
    main()
