"""Whole solves at the full sizes of the workloads, in the configuration bench.py times.

* 2D n = 2048 (4,190,209 DOF), zeta = 100: lambda against the oracle's converged discrete
  eigenvalue of (2.4) and u at 256 seeded nodes against the oracle's converged eigenvector
  (tests/golden/large_2d.json, written by make_golden.py from oracle/ only), FP64 and mixed.
* 3D 256^3 (16,581,375 DOF), zeta = 10: no oracle run reaches this size, so properties that
  hold at any size: FP64 and mixed precision agree, b(u,u) = 1, lambda equals the
  Rayleigh quotient, int u > 0, and lambda converges at second order in h (P1 elements)
  over 64^3, 128^3, 256^3.
* The batched workload at full size (64 uneven instances up to n = 1024): every instance
  bit for bit equal to its own fmg_solve."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "large_2d.json")))["large_2d"]


def _solve(prob, opts):
    from paper_1502_04657_amd import Solver
    return Solver(prob, opts).solve()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_n2048_matches_oracle_converged_solution(precision):
    res, u = _solve(W.LARGE_2D, W.Options(tol_lambda=1e-12, max_final_steps=100, precision=precision))
    assert res.status == 0
    lam_ref = GOLD["lambda_ref"]
    assert abs(res.lam - lam_ref) <= 1e-10 * lam_ref
    idx = torch.tensor(GOLD["sample_index"], device="cuda")
    got = u[idx].cpu().numpy()
    want = np.asarray(GOLD["sample_u"])
    s = np.sign(got @ want)
    assert np.abs(s * got - want).max() <= 1e-8 * np.abs(want).max()
    assert res.norm == pytest.approx(1.0, abs=1e-12)
    assert res.lambda_rq == pytest.approx(res.lam, rel=1e-11)


def _m_norm_diff(prob, u1, u2):
    from paper_1502_04657_amd import ops
    n = prob.n_coarse << prob.n_refine
    d = ops.pack(prob.dim, n, (u1 - u2).contiguous())
    return float(np.sqrt(max(ops.forms(prob, n, d)[2], 0.0)))


def test_3d_256_mixed_matches_fp64_and_identities():
    prob = W.LARGE_3D
    r64, u64 = _solve(prob, W.Options(tol_lambda=1e-11, max_final_steps=100))
    rmx, umx = _solve(prob, W.Options(tol_lambda=1e-11, max_final_steps=100, precision="mixed"))
    for r in (r64, rmx):
        assert r.status == 0
        assert r.norm == pytest.approx(1.0, abs=1e-11)
        assert r.lambda_rq == pytest.approx(r.lam, rel=1e-10)
    assert abs(r64.lam - rmx.lam) <= 1e-10 * r64.lam
    assert _m_norm_diff(prob, u64, umx) <= 1e-7
    assert float(u64.sum()) > 0 and float(umx.sum()) > 0


def test_3d_eigenvalue_converges_at_second_order():
    lams = []
    for refine in (4, 5, 6):   # n = 64, 128, 256 from the 4^3 coarsest mesh
        prob = W.Problem(3, 4, refine, (1.0, 1.0, 1.0), 0.0, 10.0)
        r, _ = _solve(prob, W.Options(tol_lambda=1e-11, max_final_steps=100))
        assert r.status == 0
        lams.append(r.lam)
    ratio = (lams[0] - lams[1]) / (lams[1] - lams[2])
    assert 3.5 < ratio < 4.5, (lams, ratio)
    assert lams[0] > lams[1] > lams[2]   # conforming P1: the discrete lambda decreases under refinement


def test_batched_workload_matches_solo_bitwise():
    from paper_1502_04657_amd import Solver, batch_solve
    probs = W.batch_instances(64, 0)
    opts = W.Options(tol_lambda=1e-9, precision="mixed")
    res, us = batch_solve(probs, opts, check=False)
    for p, r, u in zip(probs, res, us):
        s, su = Solver(p, opts).solve(check=False)
        assert r.status == s.status
        assert r.lam == s.lam and r.history == s.history
        assert torch.equal(u, su)
