"""Geometric multigrid for the auxiliary boundary-value problem (3.4), used as the
MG(V_{h_k}, rhs, u0, m) of (3.5).

The paper leaves the cycle and the smoother open (its experiments use 3 CG smoothing
steps).  The reading implemented here, shared with the HIP library by specification
only: a V(nu_pre, nu_post) cycle whose smoother is symmetric Gauss-Seidel in red-black
order (red = (i+j[+k]) even): one SGS sweep is a forward pass (red, then black) followed
by a backward pass (black, then red).  The smoother of the paper's experiments is
available too: nu_pre / nu_post steps of the plain conjugate gradient method on K_l x = f
started from the current x (the cycle is then a nonlinear, variable preconditioner).
Level operators are the rediscretised stiffness matrices (equal to the Galerkin products
P^T K P, checked in the tests), transfers are P1 interpolation and its transpose, and the
coarsest level is solved exactly (dense Cholesky).  There is no damping.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem
from .mesh import Mesh, interior_parity


class Level:
    def __init__(self, mesh: Mesh, K: sp.csr_matrix):
        self.mesh, self.K = mesh, K
        self.diag = K.diagonal()
        par = interior_parity(mesh.dim, mesh.n)
        self.red, self.black = par == 0, par == 1
        for mask in (self.red, self.black):
            blk = K[mask][:, mask]
            off = blk - sp.diags(blk.diagonal())
            # Gauss-Seidel inside one colour equals a simultaneous update only because
            # no two nodes of the same colour are coupled; check that this holds.
            assert off.count_nonzero() == 0 or np.abs(off.data).max() < 1e-14 * np.abs(self.diag).max()


def gs_half_sweep(lv: Level, x: np.ndarray, f: np.ndarray, mask: np.ndarray) -> None:
    """x_i <- (f_i - sum_{j != i} K_ij x_j) / K_ii for every node i of one colour."""
    r = f - lv.K @ x
    x[mask] += r[mask] / lv.diag[mask]


def sgs_sweep(lv: Level, x, f) -> None:
    """One symmetric Gauss-Seidel sweep: forward (red, black), backward (black, red)."""
    gs_half_sweep(lv, x, f, lv.red)
    gs_half_sweep(lv, x, f, lv.black)
    gs_half_sweep(lv, x, f, lv.black)
    gs_half_sweep(lv, x, f, lv.red)


def cg_steps(lv: Level, x: np.ndarray, f: np.ndarray, steps: int) -> None:
    """`steps` iterations of the conjugate gradient method for K x = f from x (in place):
    r = f - K x, p = r; per step q = K p, alpha = (r.r)/(p.q), x += alpha p,
    r -= alpha q, beta = (r'.r')/(r.r), p = r' + beta p.  Stops early on r = 0."""
    r = f - lv.K @ x
    p = r.copy()
    rr = float(r @ r)
    for _ in range(steps):
        if rr == 0.0:
            return
        q = lv.K @ p
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new


def smooth(lv: Level, x, f, nu: int, smoother: str) -> None:
    if smoother == "cg":
        cg_steps(lv, x, f, nu)
        return
    for _ in range(nu):
        sgs_sweep(lv, x, f)


def gs_sequential(K: sp.csr_matrix, x, f, order) -> None:
    """Textbook Gauss-Seidel visiting the dofs one by one in the given order (tiny cases)."""
    Kd = K.toarray()
    for i in order:
        x[i] = (f[i] - Kd[i] @ x + Kd[i, i] * x[i]) / Kd[i, i]


class MGHierarchy:
    """Levels 0..L-1 (level 0 = coarsest) with prolongations P[l]: level l-1 -> l."""

    def __init__(self, dim: int, n_coarse: int, n_levels: int, meshes=None, stiff=None):
        self.meshes = meshes or [Mesh(dim, n_coarse << l) for l in range(n_levels)]
        Ks = stiff or [fem.stiffness(m) for m in self.meshes]
        self.levels = [Level(m, K) for m, K in zip(self.meshes, Ks)]
        self.P = [None] + [fem.prolongation(self.meshes[l], self.meshes[l - 1])
                           for l in range(1, n_levels)]
        self.coarse_chol = sla.cho_factor(Ks[0].toarray())

    def coarse_solve(self, f):
        return sla.cho_solve(self.coarse_chol, f)

    def vcycle(self, l: int, x: np.ndarray, f: np.ndarray, nu_pre: int, nu_post: int,
               smoother: str = "sgs") -> np.ndarray:
        """One V(nu_pre, nu_post) cycle for K_l x = f; returns the new x."""
        if l == 0:
            return self.coarse_solve(f)
        lv = self.levels[l]
        x = x.copy()
        smooth(lv, x, f, nu_pre, smoother)
        r = f - lv.K @ x
        rc = self.P[l].T @ r
        ec = self.vcycle(l - 1, np.zeros_like(rc), rc, nu_pre, nu_post, smoother)
        x += self.P[l] @ ec
        smooth(lv, x, f, nu_post, smoother)
        return x

    def mg(self, l: int, f: np.ndarray, x0: np.ndarray, m: int, nu_pre: int, nu_post: int,
           smoother: str = "sgs"):
        """MG(V_l, f, x0, m) of (3.5): m V-cycles started from x0."""
        x = x0
        for _ in range(m):
            x = self.vcycle(l, x, f, nu_pre, nu_post, smoother)
        return x
