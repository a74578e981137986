"""GPU parity of whole FMG eigensolves (Algorithm 3.2) through fmg_solve against the
oracle's stored results (tests/golden/small.json, written by make_golden.py from oracle/
only):
  * fixed schedule, FP64: the lambda after every correction step equals the oracle's
    (same algorithm, only rounding differs) and so does u;
  * converged (tolerance mode), FP64 and mixed precision: lambda within 1e-10 relative and
    u within 1e-8 in the M-norm of the converged discrete solution of (2.4);
  * identities on every result: b(u,u) = 1, lambda = a(u,u)/b(u,u), int u > 0."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import oracle_hierarchy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small.json")))


def _problem(rec):
    p = rec["problem"]
    return W.Problem(p["dim"], p["n_coarse"], p["n_refine"], tuple(p["w_quad"]), p["w_const"], p["zeta"],
                     tuple(p.get("diffusion", (1.0, 1.0, 1.0))))


def _solve(prob, opts):
    from paper_1502_04657_amd import Solver
    return Solver(prob, opts).solve()


ALL = ["small_2d", "small_2d_z100", "small_3d", "small_2d_z1000", "small_3d_nc6", "small_3d_nc12", "small_3d_nc16",
       "small_2d_aniso", "small_3d_aniso"]


@pytest.mark.parametrize("name", ALL)
def test_fixed_schedule_matches_oracle_step_by_step(name):
    rec = GOLD[name]
    prob = _problem(rec)
    res, u = _solve(prob, W.Options())
    hist = rec["fixed_history"]
    assert len(res.history) == len(hist)
    for a, b in zip(res.history, hist):
        assert a == pytest.approx(b, rel=1e-11)
    h = oracle_hierarchy(prob)
    M = h.M[h.L - 1]
    d = u.cpu().numpy() - np.asarray(rec["fixed_u"])
    assert math.sqrt(d @ (M @ d)) < 1e-9
    assert res.norm == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_matches_discrete_solution(name, precision):
    rec = GOLD[name]
    prob = _problem(rec)
    opts = W.Options(tol_lambda=1e-13, max_final_steps=200, precision=precision)
    res, u = _solve(prob, opts)
    assert res.status == 0
    assert res.lam == pytest.approx(rec["lambda_ref"], rel=1e-10)
    h = oracle_hierarchy(prob)
    M = h.M[h.L - 1]
    d = u.cpu().numpy() - np.asarray(rec["u_ref"])
    assert math.sqrt(d @ (M @ d)) < 1e-8
    assert res.norm == pytest.approx(1.0, abs=1e-12)
    assert res.lambda_rq == pytest.approx(res.lam, rel=1e-11)
    assert float(h.hat(h.L - 1) @ u.cpu().numpy()) > 0


def test_tolerance_mode_reaches_1e8_error():
    rec = GOLD["small_2d_z100"]
    prob = _problem(rec)
    for precision in ("fp64", "mixed"):
        res, _ = _solve(prob, W.Options(tol_lambda=1e-9, precision=precision))
        assert res.status == 0
        assert abs(res.lam - rec["lambda_ref"]) <= 1e-8 * rec["lambda_ref"]


def test_repeat_solves_are_bitwise_identical():
    from paper_1502_04657_amd import Solver
    prob = _problem(GOLD["small_2d"])
    s = Solver(prob, W.Options(tol_lambda=1e-12))
    r1, u1 = s.solve()
    r2, u2 = s.solve()
    assert r1.lam == r2.lam
    assert torch.equal(u1, u2)
    assert r1.history == r2.history


def test_solve_reports_nonconvergence_cap():
    from paper_1502_04657_amd import FmgError, Solver
    prob = _problem(GOLD["small_2d_z1000"])
    s = Solver(prob, W.Options(tol_lambda=1e-15, max_final_steps=1))
    with pytest.raises(FmgError) as e:
        s.solve()
    assert e.value.code == -3


@pytest.mark.parametrize("fixed", [1, 2, 3])
def test_fixed_iteration_count_variant_reaches_the_same_solution(fixed):
    # a fixed number of nonlinear iterations per augmented problem (Section 3.3) changes
    # the iterates but not the fixed point of Algorithm 3.1, where u~ already solves (3.6)
    rec = GOLD["small_2d_z100"]
    prob = _problem(rec)
    conv, _ = _solve(prob, W.Options(tol_lambda=1e-13, max_final_steps=200))
    res, u = _solve(prob, W.Options(tol_lambda=1e-13, max_final_steps=200, newton_fixed_iters=fixed))
    assert res.status == 0
    assert res.lam == pytest.approx(rec["lambda_ref"], rel=1e-10)
    h = oracle_hierarchy(prob)
    M = h.M[h.L - 1]
    d = u.cpu().numpy() - np.asarray(rec["u_ref"])
    assert math.sqrt(d @ (M @ d)) < 1e-8
    assert res.newton_total < conv.newton_total


@pytest.mark.parametrize("prob", [W.Problem(3, 8, 1, (1.0, 1.0, 1.0), 0.0, 10.0),
                                  W.Problem(2, 24, 2, (1.0, 1.0, 0.0), 0.0, 30.0)])
def test_fixed_schedule_with_global_memory_small_solves_matches_oracle(prob):
    # coarsest h = 1/8 in 3D (N_H = 343, 49 x 49 blocks) and h = 1/24 in 2D (N_H = 529,
    # 23 x 23 blocks): the small-solve arena lives in global memory, the block inversions
    # go through LDS in groups, and in 2D the chord steps' per-simplex residual values use
    # global scratch
    from oracle import fmg as ofmg
    ref = ofmg.fmg(prob, W.Options(), hierarchy=oracle_hierarchy(prob))
    res, u = _solve(prob, W.Options())
    assert len(res.history) == len(ref.history)
    for a, (_, _, b) in zip(res.history, ref.history):
        assert a == pytest.approx(b, rel=1e-10)
    h = oracle_hierarchy(prob)
    d = u.cpu().numpy() - ref.u
    assert math.sqrt(d @ (h.M[h.L - 1] @ d)) < 1e-9


def test_result_reports_residual_and_contraction():
    """A converged solve has a tiny nodal residual of (2.4) and a correction-step contraction
    estimate below 1 (Theorem 3.1); a fixed schedule with p = 2 has too few finest steps."""
    rec = GOLD["small_2d_z100"]
    prob = _problem(rec)
    res, _ = _solve(prob, W.Options(tol_lambda=1e-12, max_final_steps=100))
    assert res.status == 0
    assert 0.0 <= res.residual < 1e-9
    assert 0.0 < res.gamma_est < 1.0
    fixed, _ = _solve(prob, W.Options())
    assert fixed.gamma_est == -1.0
    assert fixed.residual > res.residual


@pytest.mark.parametrize("prob", [W.Problem(3, 2, 2, (1.0, 0.5, 2.0), 0.3, 10.0),
                                  W.Problem(3, 3, 2, (1.0, 1.0, 1.0), 0.0, 30.0)])
def test_3d_result_forms_match_oracle_operators(prob):
    """The norm, Rayleigh quotient and relative nodal residual a 3D solve reports (the
    row-based forms pass over the final u; n = 8 and a ragged n = 12) against the oracle's
    operators applied to the returned u: b(u,u) = u^T M u, (a(u,u) + zeta int u^4) / b(u,u)
    with a = K + M_W, and |K u - (lambda M u - M_W u - zeta N(u))| / |lambda M u|."""
    res, u = _solve(prob, W.Options(tol_lambda=1e-9))
    assert res.status == 0
    h = oracle_hierarchy(prob)
    l = h.L - 1
    x = u.cpu().numpy()
    a_uu, b_uu, q4 = h.energy_terms(l, x)
    assert res.norm == pytest.approx(b_uu, rel=1e-12)
    assert res.lambda_rq == pytest.approx((a_uu + prob.zeta * q4) / b_uu, rel=1e-12)
    r = h.K[l] @ x - h.rhs(l, res.lam, x)
    lm = res.lam * (h.M[l] @ x)
    want = math.sqrt(float(r @ r) / float(lm @ lm))
    # the residual is a difference of terms about 1e8 times larger: rounding of either
    # side moves it by about 1e-16 / 1e-8 relative
    assert res.residual == pytest.approx(want, rel=1e-5)


def test_host_output_and_library_allocated_workspace_match_device_solve():
    from paper_1502_04657_amd import Solver, solve_alloc
    prob = _problem(GOLD["small_3d"])
    opts = W.Options(tol_lambda=1e-10)
    s = Solver(prob, opts)
    r_dev, u_dev = s.solve()
    u_host = torch.zeros(s.ndof, dtype=torch.float64)
    r_host, _ = s.solve(u_host)
    assert r_host.lam == r_dev.lam
    assert torch.equal(u_host, u_dev.cpu())
    r_a, u_a = solve_alloc(prob, opts)
    assert r_a.lam == r_dev.lam and r_a.history == r_dev.history
    assert torch.equal(u_a, u_dev)
    u_ah = torch.zeros(s.ndof, dtype=torch.float64)
    r_ah, _ = solve_alloc(prob, opts, u_out=u_ah)
    assert torch.equal(u_ah, u_dev.cpu())


@pytest.mark.parametrize("name", ["small_2d_aniso", "small_3d_aniso"])
def test_anisotropic_unfused_path_matches_oracle(name):
    """The unfused kernel sequence (every level) with A = diag(a) against the oracle's
    fixed schedule, step by step."""
    from paper_1502_04657_amd import lib
    rec = GOLD[name]
    prob = _problem(rec)
    lib().fmg_set_fused_vcycle(0)
    try:
        res, _ = _solve(prob, W.Options())
    finally:
        lib().fmg_set_fused_vcycle(1)
    for a, b in zip(res.history, rec["fixed_history"]):
        assert a == pytest.approx(b, rel=1e-11)


@pytest.mark.parametrize("prob", [W.Problem(2, 16, 5, (1.0, 0.6, 0.0), 0.0, 80.0, (0.7, 1.6, 1.0)),
                                  W.Problem(3, 4, 5, (1.2, 0.8, 1.0), 0.0, 10.0, (1.5, 0.6, 1.1))])
def test_anisotropic_fused_levels_match_unfused_bitwise(prob):
    """With A = diag(a), the fused level passes (2D wide tiles at n = 512; 3D z-pipelined
    passes at n = 128) and both one-workgroup bottoms give the bits of the unfused kernels
    over a whole solve."""
    from paper_1502_04657_amd import lib
    opts = W.Options(tol_lambda=1e-9)
    r1, u1 = _solve(prob, opts)
    lib().fmg_set_fused_vcycle(0)
    try:
        r0, u0 = _solve(prob, opts)
    finally:
        lib().fmg_set_fused_vcycle(1)
    assert r1.status == 0 and r0.status == 0
    assert r1.lam == r0.lam and r1.history == r0.history
    assert torch.equal(u1, u0)
