"""The conjugate-gradient smoother (the smoother of the paper's experiments) against the
oracle: single smoothing calls element by element, whole FMG solves with m = p = 1 and
3 + 3 CG steps step by step (fixed schedule), and converged solves against the discrete
solution of (2.4)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import dev_level, host_compact, oracle_hierarchy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small.json")))
CG = dict(m=1, p=1, nu_pre=3, nu_post=3, smoother="cg")


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 37), (3, 8), (3, 11)])
@pytest.mark.parametrize("steps", [1, 2, 3])
def test_cg_steps_match_oracle(dim, n, steps):
    from oracle.mg import Level, cg_steps
    from oracle.mesh import Mesh
    from oracle import fem
    from paper_1502_04657_amd import ops
    mesh = Mesh(dim, n)
    lv = Level(mesh, fem.stiffness(mesh))
    rng = np.random.default_rng(7 + n + steps)
    x0 = rng.standard_normal(lv.K.shape[0])
    f = rng.standard_normal(lv.K.shape[0])
    want = x0.copy()
    cg_steps(lv, want, f, steps)
    x = dev_level(dim, n, x0)
    ops.cg_smooth(dim, n, x, dev_level(dim, n, f), steps)
    got = host_compact(dim, n, x)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_cg_smoothing_of_a_solution_leaves_it():
    # r = 0 at the start: x must not move (alpha = beta = 0, as in the oracle's early exit)
    from oracle import fem
    from oracle.mesh import Mesh
    from paper_1502_04657_amd import ops
    mesh = Mesh(2, 16)
    K = fem.stiffness(mesh)
    xs = np.random.default_rng(1).standard_normal(K.shape[0])
    x = dev_level(2, 16, xs)
    ops.cg_smooth(2, 16, x, dev_level(2, 16, K @ xs), 3)
    assert np.abs(host_compact(2, 16, x) - xs).max() <= 1e-13


@pytest.mark.parametrize("prob", [W.Problem(2, 8, 2, (1.0, 1.0, 0.0), 0.0, 10.0),
                                  W.Problem(3, 4, 1, (1.0, 1.0, 1.0), 0.0, 1.0)])
def test_fixed_schedule_with_cg_smoother_matches_oracle(prob):
    from oracle import fmg as ofmg
    from paper_1502_04657_amd import Solver
    opts = W.Options(**CG)
    ref = ofmg.fmg(prob, opts, hierarchy=oracle_hierarchy(prob))
    res, u = Solver(prob, opts).solve()
    assert len(res.history) == len(ref.history)
    for a, (_, _, b) in zip(res.history, ref.history):
        assert a == pytest.approx(b, rel=1e-10)
    h = oracle_hierarchy(prob)
    d = u.cpu().numpy() - ref.u
    assert math.sqrt(d @ (h.M[h.L - 1] @ d)) < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_with_cg_smoother(precision):
    rec = GOLD["small_2d"]
    p = rec["problem"]
    prob = W.Problem(p["dim"], p["n_coarse"], p["n_refine"], tuple(p["w_quad"]), p["w_const"], p["zeta"],
                     tuple(p.get("diffusion", (1.0, 1.0, 1.0))))
    from paper_1502_04657_amd import Solver
    res, _ = Solver(prob, W.Options(tol_lambda=1e-13, max_final_steps=200, precision=precision, **CG)).solve()
    assert res.status == 0
    assert res.lam == pytest.approx(rec["lambda_ref"], rel=1e-10)
