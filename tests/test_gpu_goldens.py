"""GPU parity at the sizes where the wide V-cycle tiles and the large-level kernels run,
against oracle results stored by tests/golden/make_golden.py (which calls only oracle/):

* 2D n = 512 (coarsest h = 1/16, zeta = 100; levels above n = 256 use the wide fused tiles):
  the fixed schedule (Algorithm 3.2, m = 1, p = 2, SGS(2,2)) step by step, its u, and the
  converged discrete solution of (2.4) in FP64 and mixed precision;
* 3D n = 128 (coarsest h = 1/4, zeta = 10): the same three checks.

u is compared in the relative M-norm after sign alignment (M: the oracle's mass matrix of
the finest level); lambda relatively."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    path = os.path.join(HERE, name + ".npz")
    z = np.load(path)
    meta = json.loads(str(z["meta"]))
    p = meta["problem"]
    prob = W.Problem(p["dim"], p["n_coarse"], p["n_refine"], tuple(p["w_quad"]), p["w_const"], p["zeta"],
                     tuple(p.get("diffusion", (1.0, 1.0, 1.0))))
    unfold = (lambda v: _unfold_sym3(prob.n_fine, v)) if meta["folded_sym3"] else (lambda v: v)
    return prob, z["fixed_history"], unfold(z["fixed_u"]), float(z["lambda_ref"]), unfold(z["u_ref"])


def _unfold_sym3(n, v):
    """Inverse of the fold of make_golden.py: node (i, j, k) takes the stored value of its
    sorted index triple."""
    m = n - 1
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    keep = (i <= j) & (j <= k)
    table = np.full((m, m, m), np.nan)
    table[keep] = v
    s = np.sort(np.stack([i, j, k], axis=-1), axis=-1)     # ascending: (a, b, c), a <= b <= c
    out = table[s[..., 2], s[..., 1], s[..., 0]]            # table is indexed [k, j, i] with i <= j <= k
    assert not np.isnan(out).any()
    return out.ravel()


_MASS = {}


def _mass(prob):
    if prob not in _MASS:
        from oracle import fem
        from oracle.mesh import Mesh
        _MASS[prob] = fem.mass(Mesh(prob.dim, prob.n_fine))
    return _MASS[prob]


def _rel_m(prob, got, want):
    M = _mass(prob)
    s = 1.0 if got @ (M @ want) >= 0 else -1.0
    d = s * got - want
    return math.sqrt(d @ (M @ d)) / math.sqrt(want @ (M @ want))


def _solve(prob, opts):
    from paper_1502_04657_amd import Solver
    r, u = Solver(prob, opts).solve()
    return r, u.cpu().numpy()


@pytest.mark.parametrize("name", ["mid_2d", "mid_3d"])
def test_fixed_schedule_step_by_step(name):
    prob, hist, u_fixed, _, _ = _load(name)
    res, u = _solve(prob, W.Options())
    assert res.status == 0
    assert len(res.history) == len(hist)
    for a, b in zip(res.history, hist):
        assert a == pytest.approx(b, rel=1e-11)
    assert _rel_m(prob, u, u_fixed) <= 1e-9


@pytest.mark.parametrize("name", ["mid_2d", "mid_3d"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_solution(name, precision):
    prob, _, _, lam_ref, u_ref = _load(name)
    res, u = _solve(prob, W.Options(tol_lambda=1e-13, max_final_steps=200, precision=precision))
    assert res.status == 0
    assert abs(res.lam - lam_ref) <= 1e-10 * lam_ref
    assert _rel_m(prob, u, u_ref) <= 1e-8
