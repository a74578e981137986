"""Writes the stored expected values of the GPU tests and the benchmark.  Calls only the
oracle (oracle/), never the HIP library.

    python tests/golden/make_golden.py small     # seconds: fixed-schedule and converged
                                                  # results of the small workloads
    python tests/golden/make_golden.py large_2d   # long (tens of minutes): converged
                                                  # lambda of the 2D 4.2M-dof workload
    python tests/golden/make_golden.py mid_2d     # minutes: 2D n = 512 (wide V-cycle tiles),
                                                  # fixed-schedule history and u, converged u
    python tests/golden/make_golden.py large_3d   # long (about an hour): 3D 128^3, fixed-
                                                  # schedule history and u, converged u

Each JSON file holds, per workload: the problem, the oracle's fixed-schedule lambda history
(Algorithm 3.2 with m = 1, p = 2, SGS(2,2)), the converged discrete eigenvalue lambda_ref
of (2.4) on the finest level, its eigenvector at seeded sample nodes, and ||u||_M
(= 1) with int u^4 for cross-checks.
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import fem, fmg  # noqa: E402

SMALL = {
    "small_2d": W.SMALL_2D,
    "small_2d_z100": W.Problem(2, 16, 2, (1.0, 1.0, 0.0), 0.0, 100.0),
    "small_2d_z1000": W.Problem(2, 16, 2, (0.7, 1.6, 0.0), 0.0, 1000.0),
    "small_3d": W.Problem(3, 4, 2, (1.0, 1.0, 1.0), 0.0, 10.0),
    # coarsest h = 1/6: 25 x 25 coarse blocks, the largest 3D coarse space whose small-solve
    # arena fits in LDS
    "small_3d_nc6": W.Problem(3, 6, 2, (1.0, 1.0, 1.0), 0.0, 30.0),
    # coarsest h = 1/12 (N_H = 1331): the coarse space chosen for 3D n = 192 at large zeta
    "small_3d_nc12": W.Problem(3, 12, 1, (0.8, 1.3, 1.7), 0.0, 300.0),
    # coarsest h = 1/16 (N_H = 3375): the coarse space chosen for 3D n = 64 and 128 at the
    # largest zeta of the serving mix (zeta H^2 = 3.1)
    "small_3d_nc16": W.Problem(3, 16, 1, (1.3, 0.6, 1.9), 0.0, 800.0),
    # a constant diagonal coefficient A = diag(diffusion) in a-hat (2.5)
    "small_2d_aniso": W.Problem(2, 8, 3, (1.2, 0.7, 0.0), 0.3, 40.0, (0.6, 1.7, 1.0)),
    "small_3d_aniso": W.Problem(3, 4, 2, (0.9, 1.3, 1.1), 0.0, 25.0, (1.4, 0.5, 0.9)),
}
BATCH4_PICKS = (62, 22)
# Arrays too large for JSON go to compressed .npz files next to it.
MID_2D = W.Problem(2, 16, 5, (1.0, 1.0, 0.0), 0.0, 100.0)        # n = 512
MID_3D = W.Problem(3, 4, 5, (1.0, 1.0, 1.0), 0.0, 10.0)          # n = 128


def fold_sym3(n: int, u: np.ndarray) -> np.ndarray:
    """Values of a 3D interior vector at the nodes i <= j <= k (x-fastest compact order).
    W = x^2 + y^2 + z^2 and the Kuhn mesh are invariant under axis permutations, so the
    ground state is too; the fold is checked before it is taken."""
    m = n - 1
    a = u.reshape(m, m, m)                         # [k, j, i]
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
        asym = float(np.abs(a - a.transpose(perm)).max())
        assert asym <= 1e-12 * float(np.abs(a).max()), asym
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    keep = (i <= j) & (j <= k)
    return a[keep]


def run_npz(name, prob, sym3=False):
    """Fixed-schedule history and u, converged lambda_ref and u_ref, into <name>.npz."""
    t0 = time.time()
    opts = W.Options()
    h = fmg.Hierarchy(prob)
    r = fmg.fmg(prob, opts, h)
    print(f"{name}: fixed schedule lambda={r.lam:.15f} ({time.time() - t0:.1f}s)", flush=True)
    rc = fmg.converged(prob, opts, h)
    l = h.L - 1
    n = prob.n_fine
    fold = (lambda v: fold_sym3(n, v)) if sym3 else (lambda v: v)
    meta = {"problem": dataclasses.asdict(prob), "options": dataclasses.asdict(opts),
            "folded_sym3": bool(sym3), "converged_steps": int(rc.steps_total),
            "norm_M": float(rc.u @ (h.M[l] @ rc.u)), "oracle_seconds": time.time() - t0}
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, meta=json.dumps(meta), fixed_history=np.array([x[2] for x in r.history]),
                        fixed_u=fold(r.u), lambda_ref=np.array(rc.lam), u_ref=fold(rc.u))
    print(f"{name}: lambda_ref={rc.lam:.15f} steps={rc.steps_total} ({time.time() - t0:.1f}s)", flush=True)
    print("wrote", path)


def run(name, prob, fixed=True, samples=64):
    t0 = time.time()
    opts = W.Options()
    h = fmg.Hierarchy(prob)
    out = {"problem": dataclasses.asdict(prob), "options": dataclasses.asdict(opts)}
    if fixed:
        r = fmg.fmg(prob, opts, h)
        out["fixed_history"] = [float(x[2]) for x in r.history]
        out["fixed_lambda"] = float(r.lam)
        out["fixed_u"] = r.u.tolist() if r.u.size <= 40000 else None
    rc = fmg.converged(prob, opts, h)
    l = h.L - 1
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(rc.u.size, size=min(samples, rc.u.size), replace=False))
    out["lambda_ref"] = float(rc.lam)
    out["converged_steps"] = int(rc.steps_total)
    out["sample_index"] = idx.tolist()
    out["sample_u"] = rc.u[idx].tolist()
    out["norm_M"] = float(rc.u @ (h.M[l] @ rc.u))
    out["int_u4"] = float(fem.integral_of(h.meshes[l], rc.u, 4))
    out["u_ref"] = rc.u.tolist() if rc.u.size <= 40000 else None
    out["oracle_seconds"] = time.time() - t0
    print(f"{name}: lambda_ref={rc.lam:.15f} steps={rc.steps_total} ({out['oracle_seconds']:.1f}s)", flush=True)
    return out


def main(which, only=None):
    if which == "small":
        path = os.path.join(HERE, "small.json")
        if only:
            # recompute the named entries only, keeping the others as stored
            res = json.load(open(path))
            for k in only:
                res[k] = run(k, SMALL[k])
        else:
            res = {k: run(k, p) for k, p in SMALL.items()}
    elif which == "mid_2d":
        run_npz("mid_2d", MID_2D)
        return
    elif which == "large_3d":
        run_npz("mid_3d", MID_3D, sym3=True)
        return
    elif which == "large_2d":
        res = {"large_2d": run("large_2d", W.LARGE_2D, fixed=False, samples=256)}
        path = os.path.join(HERE, "large_2d.json")
    elif which == "batch4":
        # two instances of the seeded batched workload (64 instances, seed 0): the largest
        # zeta at n = 256 and at n = 512; converged lambda and u into batch4.npz
        inst = W.batch_instances(64, 0)
        arrays = {}
        for k in BATCH4_PICKS:
            t0 = time.time()
            prob = inst[k]
            rc = fmg.converged(prob, W.Options(), fmg.Hierarchy(prob))
            arrays[f"u_ref_{k}"] = rc.u
            arrays[f"lambda_ref_{k}"] = np.float64(rc.lam)
            arrays[f"meta_{k}"] = np.array(json.dumps({"problem": dataclasses.asdict(prob), "instance": k,
                                                       "converged_steps": int(rc.steps_total),
                                                       "oracle_seconds": time.time() - t0}))
            print(f"batch4_{k}: lambda_ref={rc.lam:.15f} ({time.time() - t0:.1f}s)", flush=True)
        np.savez_compressed(os.path.join(HERE, "batch4.npz"), **arrays)
        return
    else:
        raise SystemExit(f"unknown set {which}")
    with open(path, "w") as f:
        json.dump(res, f)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "small", sys.argv[2:])
