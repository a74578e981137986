"""Degenerate and boundary cases of the method on the GPU path, each against the oracle:
  * zeta = 0 (the linear eigenproblem): the converged lambda and u equal the lowest
    eigenpair of the dense generalised problem (K + M_W) u = lambda M u;
  * a single level (n_refine = 0): the solve is Algorithm 3.2 step 1 alone;
  * the smallest coarsest mesh (2D h = 1/2: one coarse unknown, 1 x 1 blocks);
  * a ragged finest level in 3D (n - 1 = 47 nodes per side against the 3D kernels)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from tests.gpu_util import oracle_hierarchy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(prob, opts):
    from paper_1502_04657_amd import Solver
    return Solver(prob, opts).solve()


@pytest.mark.parametrize("prob", [W.Problem(2, 8, 2, (1.0, 1.0, 0.0), 0.0, 0.0),
                                  W.Problem(2, 4, 3, (0.0, 0.0, 0.0), 0.0, 0.0),
                                  W.Problem(3, 4, 1, (1.0, 2.0, 0.5), 0.0, 0.0)])
def test_zeta_zero_is_the_linear_ground_state(prob):
    h = oracle_hierarchy(prob)
    l = h.L - 1
    A = (h.K[l] + h.MW[l]).toarray()
    M = h.M[l].toarray()
    w, v = sla.eigh(A, M, subset_by_index=[0, 0])
    # a long fixed schedule: once lambda has converged to rounding, a |dlambda| test cannot
    # resolve eigenvector errors much below sqrt(eps), so the vector is converged by steps
    res, u = _solve(prob, W.Options(p=40))
    assert res.status == 0
    assert res.lam == pytest.approx(float(w[0]), rel=1e-10)
    x = v[:, 0] / math.sqrt(v[:, 0] @ M @ v[:, 0])
    x *= np.sign(x.sum())
    d = u.cpu().numpy() - x
    assert math.sqrt(d @ M @ d) < 1e-8


@pytest.mark.parametrize("prob", [W.Problem(2, 16, 0, (1.0, 1.0, 0.0), 0.0, 100.0),
                                  W.Problem(3, 4, 0, (1.0, 1.0, 1.0), 0.0, 10.0)])
def test_single_level_is_the_coarse_nonlinear_solve(prob):
    from oracle import fmg as ofmg
    h = oracle_hierarchy(prob)
    lam, x, _ = ofmg.coarse_step(h)
    res, u = _solve(prob, W.Options())
    assert res.status == 0 and res.levels == 1
    assert res.lam == pytest.approx(lam, rel=1e-11)
    d = u.cpu().numpy() - x
    assert math.sqrt(d @ (h.M[0] @ d)) < 1e-10


@pytest.mark.parametrize("prob", [W.Problem(2, 2, 4, (1.0, 1.0, 0.0), 0.0, 1.0),
                                  W.Problem(3, 3, 4, (1.0, 1.0, 1.0), 0.0, 1.0)])
def test_smallest_and_ragged_coarse_meshes_match_oracle(prob):
    from oracle import fmg as ofmg
    ref = ofmg.fmg(prob, W.Options(), hierarchy=oracle_hierarchy(prob))
    res, u = _solve(prob, W.Options())
    assert len(res.history) == len(ref.history)
    for a, (_, _, b) in zip(res.history, ref.history):
        assert a == pytest.approx(b, rel=1e-10)
    h = oracle_hierarchy(prob)
    d = u.cpu().numpy() - ref.u
    assert math.sqrt(d @ (h.M[h.L - 1] @ d)) < 1e-9
