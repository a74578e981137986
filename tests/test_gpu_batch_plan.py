"""Batch plans (fmg_batch_plan_*): each instance's kernel sequence captured once into HIP
graphs and replayed.  Every replay must give the bits of fmg_solve on the same problem and
options (same kernels in the same order), also after other device work between replays,
and the instances run concurrently on the plan's streams."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

INSTANCES = [
    (W.Problem(2, 8, 4, (1.0, 1.0, 0.0), 0.0, 1.0), W.Options(tol_lambda=1e-9)),
    (W.Problem(2, 16, 4, (0.6, 1.7, 0.0), 0.0, 500.0), W.Options(tol_lambda=1e-9, precision="mixed")),
    (W.Problem(2, 16, 3, (1.2, 0.8, 0.0), 0.0, 30.0), W.Options()),                      # fixed schedule
    (W.Problem(3, 4, 3, (1.0, 1.0, 1.0), 0.0, 10.0), W.Options(tol_lambda=1e-9)),
    (W.Problem(3, 6, 2, (0.9, 1.4, 1.1), 0.0, 60.0), W.Options(tol_lambda=1e-9, precision="mixed")),
    (W.Problem(2, 16, 5, (1.0, 1.0, 0.0), 0.0, 100.0), W.Options(tol_lambda=1e-9)),        # wide fused tiles
]


def _solo(prob, opts):
    from paper_1502_04657_amd import Solver
    r, u = Solver(prob, opts).solve()
    return r, u.clone()


def test_plan_replays_are_bitwise_fmg_solve():
    from paper_1502_04657_amd import BatchPlan
    ref = [_solo(p, o) for p, o in INSTANCES]
    with BatchPlan([p for p, _ in INSTANCES], [o for _, o in INSTANCES]) as plan:
        for rep in range(3):
            res, us = plan.run()
            for i, ((r0, u0), r, u) in enumerate(zip(ref, res, us)):
                assert r.status == 0, (rep, i)
                assert r.lam == r0.lam and r.steps_total == r0.steps_total, (rep, i)
                assert r.lambda_rq == r0.lambda_rq and r.residual == r0.residual, (rep, i)
                assert torch.equal(u, u0), (rep, i)
            # other device work between replays: eager kernels of the library and of torch
            a = torch.randn(512, 512, device="cuda", dtype=torch.float64)
            _ = float((a @ a).sum())
            _solo(*INSTANCES[rep % len(INSTANCES)])
            torch.cuda.synchronize()


def test_plan_reports_per_instance_failures():
    """A solve that cannot meet its tolerance in the allowed steps fails alone: the others
    still finish with the bits of fmg_solve."""
    from paper_1502_04657_amd import BatchPlan
    bad = (W.Problem(2, 16, 3, (1.0, 1.0, 0.0), 0.0, 100.0), W.Options(tol_lambda=1e-15, max_final_steps=1))
    good = INSTANCES[0]
    r0, u0 = _solo(*good)
    with BatchPlan([bad[0], good[0]], [bad[1], good[1]]) as plan:
        res, us = plan.run(check=False)
    assert res[0].status != 0
    assert res[1].status == 0 and res[1].lam == r0.lam and torch.equal(us[1], u0)


def test_batched_workload_instances_match_oracle():
    """Two instances of the seeded batched workload (64 instances, seed 0; the largest zeta
    at n = 256, 447, and at n = 512, 625), solved together in one batch plan in mixed
    precision to convergence, against the oracle's converged discrete solutions
    (tests/golden/batch4.npz, written by make_golden.py from oracle/ only): lambda within
    1e-10 relative, u within 1e-8 in the relative M-norm after sign alignment."""
    from oracle import fem
    from oracle.mesh import Mesh
    from paper_1502_04657_amd import BatchPlan
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "batch4.npz"))
    picks = sorted(int(k.split("_")[-1]) for k in z.files if k.startswith("meta_"))
    inst = W.batch_instances(64, 0)
    probs = [inst[k] for k in picks]
    for k, p in zip(picks, probs):
        meta = json.loads(str(z[f"meta_{k}"]))
        assert meta["problem"]["zeta"] == p.zeta and meta["problem"]["n_refine"] == p.n_refine
    opts = W.Options(tol_lambda=1e-13, max_final_steps=200, precision="mixed")
    with BatchPlan(probs, opts) as plan:
        res, us = plan.run()
    for k, p, r, u in zip(picks, probs, res, us):
        lam_ref = float(z[f"lambda_ref_{k}"])
        want = z[f"u_ref_{k}"]
        assert r.status == 0
        assert abs(r.lam - lam_ref) <= 1e-10 * lam_ref, k
        M = fem.mass(Mesh(p.dim, p.n_fine))
        got = u.cpu().numpy()
        s = 1.0 if got @ (M @ want) >= 0 else -1.0
        d = s * got - want
        assert math.sqrt(d @ (M @ d)) <= 1e-8 * math.sqrt(want @ (M @ want)), k
