"""Pins for oracle.mg: the red-black Gauss-Seidel smoother is Gauss-Seidel, and the
V-cycle behaves as a multigrid method for the auxiliary problem (3.4)-(3.5) must:
an h-independent contraction theta < 1 (the assumption (3.7)) and convergence to the
direct solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from oracle.mesh import Mesh, interior_parity
from oracle.mg import Level, MGHierarchy, gs_half_sweep, gs_sequential, sgs_sweep


@pytest.mark.parametrize("dim, n", [(2, 6), (3, 4)])
def test_red_black_half_sweeps_equal_sequential_gauss_seidel(dim, n):
    m = Mesh(dim, n)
    K = fem.stiffness(m)
    lv = Level(m, K)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(m.ndof)
    x0 = rng.standard_normal(m.ndof)
    par = interior_parity(dim, n)
    order = list(np.nonzero(par == 0)[0]) + list(np.nonzero(par == 1)[0])
    xs = x0.copy()
    gs_sequential(K, xs, f, order)
    xr = x0.copy()
    gs_half_sweep(lv, xr, f, lv.red)
    gs_half_sweep(lv, xr, f, lv.black)
    assert np.allclose(xr, xs, rtol=1e-13, atol=1e-13)
    # the backward half of a symmetric sweep visits black, then red
    xs2 = xs.copy()
    gs_sequential(K, xs2, f, order[::-1])
    xr2 = xr.copy()
    gs_half_sweep(lv, xr2, f, lv.black)
    gs_half_sweep(lv, xr2, f, lv.red)
    assert np.allclose(xr2, xs2, rtol=1e-13, atol=1e-13)


def test_sgs_reduces_energy_error_monotonically():
    m = Mesh(2, 16)
    K = fem.stiffness(m)
    lv = Level(m, K)
    f = np.random.default_rng(1).standard_normal(m.ndof)
    xs = spla.spsolve(K.tocsc(), f)
    x = np.zeros_like(f)
    e_prev = np.inf
    for _ in range(5):
        sgs_sweep(lv, x, f)
        e = (x - xs) @ (K @ (x - xs))
        assert e < e_prev
        e_prev = e


@pytest.mark.parametrize("dim, nc, levels, bound", [(2, 4, 4, 0.15), (2, 4, 5, 0.15),
                                                     (3, 2, 3, 0.25), (3, 2, 4, 0.25)])
def test_vcycle_contraction_is_small_and_level_independent(dim, nc, levels, bound):
    H = MGHierarchy(dim, nc, levels)
    lv = H.levels[-1]
    f = np.random.default_rng(2).standard_normal(lv.mesh.ndof)
    xs = spla.spsolve(lv.K.tocsc(), f)
    x = np.zeros_like(f)
    rates = []
    for _ in range(6):
        xn = H.vcycle(levels - 1, x, f, 2, 2)
        e0, e1 = x - xs, xn - xs
        rates.append(np.sqrt(e1 @ (lv.K @ e1) / (e0 @ (lv.K @ e0))))
        x = xn
    assert max(rates) < bound
    x = np.zeros_like(f)
    for _ in range(20):
        x = H.vcycle(levels - 1, x, f, 2, 2)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_mg_is_m_vcycles_from_the_initial_guess():
    H = MGHierarchy(2, 4, 3)
    lv = H.levels[-1]
    rng = np.random.default_rng(3)
    f, x0 = rng.standard_normal(lv.mesh.ndof), rng.standard_normal(lv.mesh.ndof)
    x = H.vcycle(2, H.vcycle(2, x0, f, 2, 2), f, 2, 2)
    assert np.array_equal(H.mg(2, f, x0, 2, 2, 2), x)
    # linearity: MG(f, x0) = x0 + MG(f - K x0, 0)   (the form used by refinement loops)
    e = H.mg(2, f - lv.K @ x0, np.zeros_like(f), 1, 2, 2)
    assert np.allclose(H.mg(2, f, x0, 1, 2, 2), x0 + e, rtol=1e-12, atol=1e-12)


def test_coarse_solve_is_exact():
    H = MGHierarchy(2, 8, 2)
    K0 = H.levels[0].K
    f = np.random.default_rng(4).standard_normal(K0.shape[0])
    assert np.allclose(K0 @ H.coarse_solve(f), f, rtol=1e-13, atol=1e-13)


def test_cg_smoother_is_the_conjugate_gradient_method():
    # pinned against scipy's CG (same iterates in exact arithmetic) and against CG's finite
    # termination on a small SPD system
    import scipy.sparse.linalg as spla
    from oracle.mg import MGHierarchy, cg_steps
    h = MGHierarchy(2, 4, 2)
    lv = h.levels[1]
    rng = np.random.default_rng(3)
    f = rng.standard_normal(lv.K.shape[0])
    x0 = rng.standard_normal(lv.K.shape[0])
    for k in (1, 2, 3):
        x = x0.copy()
        cg_steps(lv, x, f, k)
        ref, _ = spla.cg(lv.K, f, x0=x0.copy(), rtol=0.0, atol=0.0, maxiter=k)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    x = x0.copy()
    cg_steps(lv, x, f, lv.K.shape[0])
    assert np.abs(lv.K @ x - f).max() <= 1e-9 * np.abs(f).max()


def test_cg_smoothed_vcycle_contracts():
    from oracle.mg import MGHierarchy
    h = MGHierarchy(3, 2, 3)
    l = 2
    K = h.levels[l].K
    rng = np.random.default_rng(4)
    xs = rng.standard_normal(K.shape[0])
    f = K @ xs
    x = np.zeros_like(f)
    errs = []
    for _ in range(4):
        x = h.vcycle(l, x, f, 3, 3, "cg")
        errs.append(np.linalg.norm(x - xs))
    assert errs[-1] < 1e-3 * np.linalg.norm(xs)
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))
