"""Solution of the small nonlinear eigenproblems of the method.

Two nonlinear eigenproblems appear:
  * Algorithm 3.2 step 1, the problem on the coarsest space V_{h_1};
  * Algorithm 3.1 step 2, the augmented problem (3.6) on V_{H,h_k} = V_H + span{u~}.
In a basis Z of the space, with u = Z x, both read

    (A + zeta S(x)) x = mu B x,   x^T B x = 1,   S(x) = Z^T M_{(Zx)^2} Z,

A = Z^T (K + M_W) Z,  B = Z^T M Z.  The paper allows a self-consistent or a Newton-type
iteration (Section 3.3).  A plain self-consistent iteration contracts too slowly for
zeta >= 100 and fails at zeta = 1000 on these meshes, so the oracle uses Newton's method
on the bordered system

    F(x, mu) = [ (A + zeta S(x)) x - mu B x ;  (1 - x^T B x) / 2 ] = 0,
    J        = [ A + 3 zeta S(x) - mu B ,  -B x ;  -(B x)^T , 0 ]

(d/dx of S(x) x is 3 S(x) because the nonlinearity is cubic), each step a dense LU solve
of the bordered matrix.  On the coarsest space, where no good start exists, zeta is raised from a small
value to its target in geometric stages (continuation), each stage started from the
previous solution.  Every result is certified to be the ground state (mu equals the
LOWEST eigenvalue of the pencil (A + zeta S(x), B), computed by a dense generalised
eigensolver).  A plain mixing SCF is kept for cross-checks at small zeta.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def lowest_eigpair(H: np.ndarray, B: np.ndarray):
    """Lowest eigenvalue and B-normalised eigenvector of the symmetric-definite pencil."""
    w, v = sla.eigh(H, B, subset_by_index=[0, 0])
    x = v[:, 0]
    return float(w[0]), x / np.sqrt(x @ B @ x)


def residual(A, B, S, zeta, x, mu) -> float:
    """||(A + zeta S) x - mu B x|| / (|mu| ||B x||)."""
    Bx = B @ x
    return float(np.linalg.norm((A + zeta * S) @ x - mu * Bx) / (abs(mu) * np.linalg.norm(Bx)))


def newton(A, B, S_of_x, zeta, x, mu=None, tol=1e-13, max_iter=40):
    """Newton on F(x, mu) = 0, each step a dense LU solve of the whole bordered Jacobian.
    Returns (mu, x, iterations) or None when it does not converge."""
    A = np.asarray(A); B = np.asarray(B)
    n = A.shape[0]
    x = x / np.sqrt(x @ B @ x)
    S = S_of_x(x)
    if mu is None:
        mu = float(x @ (A + zeta * S) @ x)
    Jb = np.zeros((n + 1, n + 1))
    for it in range(max_iter + 1):
        Bx = B @ x
        F1 = (A + zeta * S) @ x - mu * Bx
        F2 = 0.5 * (1.0 - x @ Bx)
        if np.linalg.norm(F1) <= tol * abs(mu) * np.linalg.norm(Bx) and abs(F2) <= 1e-15:
            return mu, x, it
        if it == max_iter or not np.all(np.isfinite(F1)):
            return None
        Jb[:n, :n] = A + 3.0 * zeta * S - mu * B
        Jb[:n, n] = -Bx
        Jb[n, :n] = -Bx
        Jb[n, n] = 0.0
        try:
            step = np.linalg.solve(Jb, -np.concatenate([F1, [F2]]))
        except np.linalg.LinAlgError:
            return None
        x = x + step[:n]
        mu = mu + step[n]
        S = S_of_x(x)
    return None


def newton_ground_state(A, B, S_of_x, zeta, x0, tol=1e-13, max_rounds=50):
    """Newton from x0, certified to end in the ground state.  When Newton fails or lands on
    an excited state, one self-consistent step (lowest eigenpair of the current
    Hamiltonian) is taken and Newton is restarted from there."""
    A = np.asarray(A); B = np.asarray(B)
    x = x0 / np.sqrt(x0 @ B @ x0)
    total = 0
    for _ in range(max_rounds):
        r = newton(A, B, S_of_x, zeta, x, None, tol=tol)
        if r is not None:
            mu, y, it = r
            total += it
            if is_ground_state(A, B, S_of_x, zeta, y, mu):
                return mu, y, total
        _, y = lowest_eigpair(A + zeta * S_of_x(x), B)
        x = y if y @ B @ x >= 0 else -y
        total += 1
    raise RuntimeError("no certified ground state")


def is_ground_state(A, B, S_of_x, zeta, x, mu, rtol=1e-9) -> bool:
    """True when mu is the lowest eigenvalue of (A + zeta S(x), B)."""
    lo, _ = lowest_eigpair(np.asarray(A) + zeta * S_of_x(x), np.asarray(B))
    return abs(lo - mu) <= rtol * abs(mu)


def ground_state_continuation(A, B, S_of_x, zeta, zeta_start=1.0, factor=4.0, tol=1e-13):
    """Coarse-space ground state by zeta-continuation.

    Stage values zeta_j = zeta / factor^(J-j), j = 0..J, with J the smallest integer such
    that zeta_0 <= zeta_start; stage 0 starts from the linear ground state of (A, B).
    A stage that fails is retried with the step in log(zeta) halved."""
    A = np.asarray(A); B = np.asarray(B)
    _, x = lowest_eigpair(A, B)
    if zeta == 0.0:
        mu, x = lowest_eigpair(A, B)
        return mu, x, 0
    J = max(0, math.ceil(math.log(zeta / zeta_start) / math.log(factor))) if zeta > zeta_start else 0
    log_cur = None
    log_target = math.log(zeta)
    step = math.log(factor)
    log_next = log_target - J * step
    total = 0
    mu = None
    while True:
        z = math.exp(log_next) if log_next < log_target else zeta
        r = newton(A, B, S_of_x, z, x, None, tol=tol)
        if r is None:
            if log_cur is None:
                raise RuntimeError("continuation failed at its first stage")
            step *= 0.5
            if step < 1e-3:
                raise RuntimeError("continuation step underflow")
            log_next = log_cur + step
            continue
        mu, x, it = r
        total += it
        if z == zeta:
            break
        log_cur = log_next
        log_next = min(log_target, log_cur + step)
    if not is_ground_state(A, B, S_of_x, zeta, x, mu):
        raise RuntimeError("coarse continuation converged to an excited state")
    return mu, x, total


def scf_mixing(A, B, S_of_x, zeta, x0, tol_mu=1e-14, tol_res=1e-12, max_iter=500, alpha=1.0):
    """Plain self-consistent iteration with linear density mixing (small zeta only).
    Returns (mu, x, iterations)."""
    A = np.asarray(A); B = np.asarray(B)
    x = x0 / np.sqrt(x0 @ B @ x0)
    S_in = S_of_x(x)
    mu_prev = None
    for it in range(1, max_iter + 1):
        mu, y = lowest_eigpair(A + zeta * S_in, B)
        if y @ B @ x < 0:
            y = -y
        S_out = S_of_x(y)
        res = residual(A, B, S_out, zeta, y, mu)
        if mu_prev is not None and abs(mu - mu_prev) <= tol_mu * abs(mu) and res <= tol_res:
            return mu, y, it
        S_in = (1.0 - alpha) * S_in + alpha * S_out
        mu_prev, x = mu, y
    raise RuntimeError("SCF did not converge")
