"""One correction step (Algorithm 3.1) and the full multigrid scheme (Algorithm 3.2) for
the Gross-Pitaevskii problem of Example 4.1: f(x, u) = W u + zeta u^3.

Readings of the paper used here (each is also stated where the HIP library implements it):
  * V_H = V_{h_1}: the coarse space of every augmented problem is the coarsest level.
  * The auxiliary problem (3.4) uses a-hat only (the stiffness matrix K); W and the cubic
    term sit in the right-hand side  b = lambda M u - M_W u - zeta N(u),  N(u)_a = int u^3 phi_a.
  * MG(V_k, b, u, m) is m V(nu_pre, nu_post)-cycles with red-black SGS smoothing, or with
    nu CG steps as the smoother (opts.smoother = "cg", the paper's experiments; see mg.py).
  * The basis of V_{H,h_k} is Z = [Pi_k, u~]: the coarsest hat functions written on level
    k (the composite P1 interpolation Pi_k) and u~; the augmented Newton starts from u = u~
    normalised.
  * Eigenvector sign: int u_h > 0.
  * Tolerance mode: after the p steps of the finest level, further correction steps run
    until |lambda_new - lambda_old| <= tol_lambda |lambda_new|.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse as sp

from . import fem, scf
from .mesh import Mesh
from .mg import MGHierarchy


class Hierarchy:
    """All levels of one problem, with operators built by generic assembly."""

    def __init__(self, problem):
        self.problem = problem
        d, nc, L = problem.dim, problem.n_coarse, problem.n_refine + 1
        self.L = L
        self.meshes = [Mesh(d, nc << l) for l in range(L)]
        self.W = fem.potential(problem.w_quad, problem.w_const)
        self.K = [fem.stiffness(m, getattr(problem, "diffusion", None)) for m in self.meshes]
        self.M = [fem.mass(m) for m in self.meshes]
        self.MW = [fem.potential_mass(m, self.W) for m in self.meshes]
        self.mg = MGHierarchy(d, nc, L, meshes=self.meshes, stiff=self.K)
        self.Pi = [sp.identity(self.meshes[0].ndof, format="csr")]
        for l in range(1, L):
            self.Pi.append((self.mg.P[l] @ self.Pi[l - 1]).tocsr())
        self.hats = [None] * L

    def hat(self, l):
        if self.hats[l] is None:
            self.hats[l] = fem.hat_integrals(self.meshes[l])
        return self.hats[l]

    def fix_sign(self, l, u):
        """Choose the sign with int u_h > 0."""
        return u if self.hat(l) @ u >= 0 else -u

    def rhs(self, l, lam, u):
        """b = lambda M u - M_W u - zeta N(u): the load of the auxiliary problem (3.4)."""
        z = self.problem.zeta
        b = lam * (self.M[l] @ u) - self.MW[l] @ u
        if z != 0.0:
            b -= z * fem.nonlinear_load(self.meshes[l], u)
        return b

    def energy_terms(self, l, u):
        """(u^T (K + M_W) u, u^T M u, int u^4) on level l."""
        return (float(u @ (self.K[l] @ u + self.MW[l] @ u)), float(u @ (self.M[l] @ u)),
                fem.integral_of(self.meshes[l], u, 4))

    def rayleigh(self, l, u):
        """a(u,u)/b(u,u) of (2.2) with f = W u + zeta u^3."""
        a, b, q = self.energy_terms(l, u)
        return (a + self.problem.zeta * q) / b


def coarse_step(h: Hierarchy):
    """Algorithm 3.2 step 1: ground state of the nonlinear problem on V_{h_1}."""
    A = (h.K[0] + h.MW[0]).toarray()
    B = h.M[0].toarray()

    def S_of_x(x):
        return fem.density_mass(h.meshes[0], x).toarray()
    mu, x, it = scf.ground_state_continuation(A, B, S_of_x, h.problem.zeta)
    return mu, h.fix_sign(0, x), it


def augmented_solve(h: Hierarchy, l: int, ut: np.ndarray):
    """Algorithm 3.1 step 2: the nonlinear eigenproblem (3.6) on V_H + span{u~}."""
    Pi = h.Pi[l]
    Z = sp.hstack([Pi, sp.csr_matrix(ut[:, None])]).tocsr()
    KW = h.K[l] + h.MW[l]
    A = (Z.T @ (KW @ Z)).toarray()
    B = (Z.T @ (h.M[l] @ Z)).toarray()
    mesh = h.meshes[l]

    def S_of_x(x):
        Mr = fem.density_mass(mesh, Z @ x)
        return (Z.T @ (Mr @ Z)).toarray()
    x0 = np.zeros(Z.shape[1])
    x0[-1] = 1.0
    zeta = h.problem.zeta
    mu, x, it = scf.newton_ground_state(A, B, S_of_x, zeta, x0)
    return mu, Z @ x, it, x


def correction_step(h: Hierarchy, l: int, lam: float, u: np.ndarray, opts):
    """(lambda, u) <- EigenMG(V_H, lambda, u, V_l, m): Algorithm 3.1."""
    b = h.rhs(l, lam, u)
    ut = h.mg.mg(l, b, u, opts.m, opts.nu_pre, opts.nu_post, getattr(opts, "smoother", "sgs"))
    mu, unew, it, _ = augmented_solve(h, l, ut)
    return mu, h.fix_sign(l, unew), it


@dataclasses.dataclass
class Result:
    lam: float
    u: np.ndarray
    history: list          # (level, step, lambda) after every correction step
    newton_iters: int
    steps_total: int
    seconds: float


def fmg(problem, opts, hierarchy: Hierarchy | None = None, extra_tol: float | None = None,
        max_final_steps: int | None = None) -> Result:
    """Algorithm 3.2.  extra_tol/max_final_steps override opts.tol_lambda/max_final_steps."""
    t0 = time.perf_counter()
    h = hierarchy or Hierarchy(problem)
    lam, u, it_tot = coarse_step(h)
    hist = [(0, 0, lam)]
    steps = 0
    tol = opts.tol_lambda if extra_tol is None else extra_tol
    cap = opts.max_final_steps if max_final_steps is None else max_final_steps
    for l in range(1, h.L):
        u = h.mg.P[l] @ u                       # u^{(0)} on level l: u_{l-1} in V_l
        for s in range(opts.p):
            lam, u, it = correction_step(h, l, lam, u, opts)
            it_tot += it; steps += 1
            hist.append((l, s + 1, lam))
        if l == h.L - 1 and tol > 0.0:
            prev = hist[-2][2] if opts.p > 1 else None
            extra = 0
            while prev is None or abs(lam - prev) > tol * abs(lam):
                if extra >= cap:
                    break
                prev = lam
                lam, u, it = correction_step(h, l, lam, u, opts)
                it_tot += it; steps += 1; extra += 1
                hist.append((l, opts.p + extra, lam))
    return Result(lam, u, hist, it_tot, steps, time.perf_counter() - t0)


def converged(problem, opts, hierarchy: Hierarchy | None = None, tol: float = 1e-14,
              tol_u: float = 1e-12, max_steps: int = 300) -> Result:
    """The discrete solution of (2.4) on the finest level (O2): correction steps continue
    until |d lambda| <= tol lambda and ||d u||_M <= tol_u, or until ||d u||_M stops
    decreasing for three steps (round-off floor)."""
    h = hierarchy or Hierarchy(problem)
    res = fmg(problem, opts, h, extra_tol=0.0)
    lam, u = res.lam, res.u
    l = h.L - 1
    M = h.M[l]
    stall = 0
    best = np.inf
    for _ in range(max_steps):
        prev, uprev = lam, u
        lam, u, it = correction_step(h, l, lam, u, opts)
        res.history.append((l, -1, lam))
        res.steps_total += 1
        d = u - uprev
        du = float(np.sqrt(abs(d @ (M @ d))))
        if abs(lam - prev) <= tol * abs(lam) and du <= tol_u:
            break
        stall = stall + 1 if du >= best else 0
        best = min(best, du)
        if stall >= 3:
            break
    if du > 1e-9:
        # Theorem 3.1 needs gamma < 1, i.e. a coarse space fine enough for this zeta.
        raise RuntimeError(f"correction steps do not contract (||du||_M = {du:.2e}); "
                           "the coarsest mesh is too coarse for this nonlinearity")
    res.lam, res.u = lam, u
    return res
