"""Pins for oracle.scf and oracle.fmg: the FMG result against brute-force dense
eigensolves of the discrete problem (2.4) on the full space, the linear limit zeta = 0
(lambda_h -> 2 pi^2 / 3 pi^2 with O(h^2) error, Assumption B1), the normalisation and
Rayleigh-quotient identities of (2.2), and Theorems 3.1-3.2 behaviour."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fem, fmg, scf
from oracle.mesh import Mesh

OPTS = W.Options()


def full_space_ground_state(problem, method="newton"):
    """Brute force on the finest mesh alone: dense matrices, no multigrid, no augmentation."""
    m = Mesh(problem.dim, problem.n_fine)
    Wf = fem.potential(problem.w_quad, problem.w_const)
    A = (fem.stiffness(m) + fem.potential_mass(m, Wf)).toarray()
    B = fem.mass(m).toarray()

    def S_of_x(x):
        return fem.density_mass(m, x).toarray()
    if problem.zeta == 0:
        mu, x = scf.lowest_eigpair(A, B)
    elif method == "mixing":
        _, x0 = scf.lowest_eigpair(A, B)
        mu, x, _ = scf.scf_mixing(A, B, S_of_x, problem.zeta, x0)
    else:
        mu, x, _ = scf.ground_state_continuation(A, B, S_of_x, problem.zeta)
    if fem.hat_integrals(m) @ x < 0:
        x = -x
    return mu, x, B


@pytest.mark.parametrize("problem", [
    W.Problem(2, 4, 1, (0.0, 0.0, 0.0), 0.0, 0.0),
    W.Problem(2, 4, 2, (1.0, 1.0, 0.0), 0.0, 1.0),
    W.Problem(2, 8, 1, (1.5, 0.7, 0.0), 0.0, 100.0),
    W.Problem(3, 2, 2, (1.0, 1.0, 1.0), 0.0, 10.0),
])
def test_converged_fmg_equals_full_space_solution(problem):
    ref_mu, ref_u, B = full_space_ground_state(problem)
    r = fmg.converged(problem, OPTS)
    assert r.lam == pytest.approx(ref_mu, rel=1e-12)
    d = r.u - ref_u
    assert math.sqrt(d @ B @ d) <= 1e-9


def test_too_coarse_space_is_reported():
    # H = 1/4 is too coarse for zeta = 100: gamma >= 1 in Theorem 3.1.
    with pytest.raises(RuntimeError, match="do not contract"):
        fmg.converged(W.Problem(2, 4, 2, (1.5, 0.7, 0.0), 0.0, 100.0), OPTS)


def test_newton_and_mixing_scf_agree():
    p = W.Problem(2, 4, 2, (1.0, 1.0, 0.0), 0.0, 1.0)
    mu_n, x_n, _ = full_space_ground_state(p, "newton")
    mu_s, x_s, B = full_space_ground_state(p, "mixing")
    assert mu_n == pytest.approx(mu_s, rel=1e-13)
    assert math.sqrt((x_n - x_s) @ B @ (x_n - x_s)) < 1e-10


def test_linear_limit_converges_to_two_pi_squared_at_second_order():
    lams = []
    for n in (8, 16, 32, 64):
        m = Mesh(2, n)
        K, M = fem.stiffness(m), fem.mass(m)
        w = spla.eigsh(K.tocsc(), k=1, M=M.tocsc(), sigma=0.0, which="LM")[0]
        lams.append(float(w[0]))
    err = [l - 2 * math.pi ** 2 for l in lams]
    assert all(e > 0 for e in err)
    ratios = [err[i] / err[i + 1] for i in range(3)]
    assert all(3.9 < r < 4.1 for r in ratios)
    assert abs((4 * lams[-1] - lams[-2]) / 3 - 2 * math.pi ** 2) < 1e-4
    # the multigrid scheme reproduces the n = 32 value
    r = fmg.converged(W.Problem(2, 8, 2, (0.0, 0.0, 0.0), 0.0, 0.0), OPTS)
    assert r.lam == pytest.approx(lams[2], rel=1e-12)


def test_linear_limit_3d():
    lams = []
    for n in (4, 8, 16):
        m = Mesh(3, n)
        w = spla.eigsh(fem.stiffness(m).tocsc(), k=1, M=fem.mass(m).tocsc(), sigma=0.0, which="LM")[0]
        lams.append(float(w[0]))
    err = [l - 3 * math.pi ** 2 for l in lams]
    assert all(3.8 < err[i] / err[i + 1] < 4.3 for i in range(2))


@pytest.mark.parametrize("dim, a, ns", [(2, (0.6, 1.7), (8, 16, 32, 64)), (3, (1.4, 0.5, 0.9), (4, 8, 16))])
def test_anisotropic_linear_limit_is_pi_squared_times_trace(dim, a, ns):
    """-div(A grad u) = lambda u with A = diag(a) on the unit cube: the lowest eigenvalue is
    pi^2 (a_1 + .. + a_d), approached from above at O(h^2) by the discrete pencil; the
    multigrid scheme reproduces the discrete value."""
    lams = []
    for n in ns:
        m = Mesh(dim, n)
        w = spla.eigsh(fem.stiffness(m, a).tocsc(), k=1, M=fem.mass(m).tocsc(), sigma=0.0, which="LM")[0]
        lams.append(float(w[0]))
    exact = math.pi ** 2 * sum(a)
    err = [l - exact for l in lams]
    assert all(e > 0 for e in err)
    assert all(3.7 < err[i] / err[i + 1] < 4.4 for i in range(len(err) - 1))
    p = W.Problem(dim, ns[0], 1, (0.0, 0.0, 0.0), 0.0, 0.0, tuple(a) + (1.0,) * (3 - dim))
    r = fmg.converged(p, OPTS)
    assert r.lam == pytest.approx(lams[1], rel=1e-11)


def test_anisotropic_problem_scales_with_the_domain():
    """With A = c I the problem on the unit cube is the isotropic one with W / c, zeta / c
    and lambda / c (divide the equation by c): lambda(c A, c W, c zeta) = c lambda(A, W, zeta)."""
    base = W.Problem(2, 8, 2, (1.0, 2.0, 0.0), 0.5, 20.0)
    c = 2.5
    scaled = W.Problem(2, 8, 2, (2.5, 5.0, 0.0), 1.25, 50.0, (c, c, c))
    r0 = fmg.converged(base, OPTS)
    r1 = fmg.converged(scaled, OPTS)
    assert r1.lam == pytest.approx(c * r0.lam, rel=1e-11)


@pytest.fixture(scope="module")
def small_run():
    p = W.Problem(2, 8, 2, (1.0, 1.0, 0.0), 0.0, 10.0)
    h = fmg.Hierarchy(p)
    return p, h, fmg.converged(p, OPTS, h)


def test_normalisation_rayleigh_quotient_and_sign(small_run):
    p, h, r = small_run
    l = h.L - 1
    assert r.u @ (h.M[l] @ r.u) == pytest.approx(1.0, abs=1e-13)
    assert h.rayleigh(l, r.u) == pytest.approx(r.lam, rel=1e-12)
    assert h.hat(l) @ r.u > 0
    # discrete equation (2.4): K u + M_W u + zeta N(u) = lambda M u
    res = h.K[l] @ r.u + h.MW[l] @ r.u + p.zeta * fem.nonlinear_load(h.meshes[l], r.u) - r.lam * (h.M[l] @ r.u)
    assert np.linalg.norm(res) <= 1e-10 * r.lam * np.linalg.norm(h.M[l] @ r.u)


def test_constant_potential_shifts_lambda(small_run):
    p, h, r = small_run
    q = W.Problem(p.dim, p.n_coarse, p.n_refine, p.w_quad, 3.0, p.zeta)
    rq = fmg.converged(q, OPTS)
    assert rq.lam == pytest.approx(r.lam + 3.0, rel=1e-12)
    d = rq.u - r.u
    assert math.sqrt(d @ h.M[-1] @ d) < 1e-9


def test_dlambda_dzeta_at_zero_is_quartic_integral():
    base = W.Problem(2, 4, 2, (1.0, 1.0, 0.0), 0.0, 0.0)
    r0 = fmg.converged(base, OPTS)
    eps = 1e-4
    l1 = fmg.converged(W.Problem(2, 4, 2, (1.0, 1.0, 0.0), 0.0, eps), OPTS).lam
    l2 = fmg.converged(W.Problem(2, 4, 2, (1.0, 1.0, 0.0), 0.0, 2 * eps), OPTS).lam
    deriv = (4 * l1 - l2 - 3 * r0.lam) / (2 * eps)          # second-order one-sided
    q = fem.integral_of(Mesh(2, 16), r0.u, 4)
    assert deriv == pytest.approx(q, rel=1e-6)


def test_correction_steps_contract_and_fmg_error_is_below_discretisation_error():
    p = W.Problem(2, 8, 3, (1.0, 1.0, 0.0), 0.0, 10.0)
    h = fmg.Hierarchy(p)
    rc = fmg.converged(p, OPTS, h)
    r = fmg.fmg(p, OPTS, h)
    # Theorem 3.2: the FMG error is far below the discretisation error of the level
    coarse = fmg.converged(W.Problem(2, 8, 2, (1.0, 1.0, 0.0), 0.0, 10.0), OPTS)
    assert abs(r.lam - rc.lam) < 0.01 * abs(coarse.lam - rc.lam)
    # Theorem 3.1: successive finest-level corrections contract
    fin = [lam for (l, s, lam) in rc.history if l == h.L - 1]
    d = [abs(fin[i + 1] - fin[i]) for i in range(len(fin) - 1)]
    big = [x for x in d if x > 1e-11 * rc.lam]
    assert len(big) >= 3
    assert all(big[i + 1] < 0.7 * big[i] for i in range(len(big) - 1))


def test_augmented_problem_keeps_the_discrete_solution_fixed(small_run):
    p, h, r = small_run
    l = h.L - 1
    mu, u, _, x = fmg.augmented_solve(h, l, r.u)
    assert mu == pytest.approx(r.lam, rel=1e-12)
    assert np.abs(x[:-1]).max() < 1e-8 and x[-1] == pytest.approx(1.0, abs=1e-8)


_LIN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "linear_eigs.json")))["values"]


@pytest.mark.parametrize("rec", _LIN, ids=lambda r: f"{r['dim']}d-n{r['n']}")
def test_generic_assembly_reproduces_stencil_eigenvalues(rec):
    """The oracle's element-by-element K and M have the lowest eigenvalue that the closed-form
    stencils give (tests/golden/linear_eigs.json, written by make_linear_eigs.py without
    the oracle)."""
    m = Mesh(rec["dim"], rec["n"])
    w = spla.eigsh(fem.stiffness(m).tocsc(), k=1, M=fem.mass(m).tocsc(), sigma=0.0, which="LM", tol=1e-14)[0]
    assert float(w[0]) == pytest.approx(rec["lambda"], rel=1e-11)


@pytest.mark.parametrize("dim, nc, refine", [(2, 8, 1), (2, 8, 3), (3, 4, 1)])
def test_fmg_linear_limit_reaches_stored_eigenvalue(dim, nc, refine):
    """zeta = 0, W = 0: the converged multigrid scheme ends at the stored linear eigenvalue."""
    n = nc << refine
    want = next(r["lambda"] for r in _LIN if r["dim"] == dim and r["n"] == n)
    r = fmg.converged(W.Problem(dim, nc, refine, (0.0, 0.0, 0.0), 0.0, 0.0), OPTS)
    assert r.lam == pytest.approx(want, rel=1e-12)
