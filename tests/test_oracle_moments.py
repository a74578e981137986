"""Pin for oracle.fem.coarse_simplex_moments, the per-coarse-simplex integrals that the
augmented problem (3.6) is assembled from.

With Z = [Pi, u~] (Pi: the coarsest hats written on the fine level, u~: a fine P1
function) and u_H = Pi x_H, every entry of the augmented matrices splits over the coarse
simplices E.  On E the coarse hats are the barycentric coordinates l_p, so

    (Z^T M Z)[a, u~]       = sum_E int_E u~ l_p                         (B1)
    (Z^T (K + M_W) Z)[a,u~] = sum_E int_E grad u~ . grad l_p + W u~ l_p   (KG + AW1)
    (Z^T (K + M_W) Z)[u~,u~] = sum_E int_E |grad u~|^2 + W u~^2           (Q + AW2)

and, with w = u_H + c u~ (c the last coefficient of x) and w^2 = u_H^2 + 2 c u_H u~ + c^2 u~^2,

    S[a, b]   = sum_E sum_rs X_r X_s int l_r l_s l_p l_q + 2c sum_r X_r T3[r,p,q] + c^2 T2[p,q]
    S[a, u~]  = sum_E sum_rs X_r X_s T3[r,s,p] + 2c sum_r X_r T2[r,p] + c^2 T1[p]
    S[u~, u~] = sum_E sum_rs X_r X_s T2[r,s] + 2c sum_r X_r T1[r] + c^2 T0

(X_r: x_H at the vertices of E, zero on the boundary; a, b: the interior coarse vertices p,
q of E).  The test assembles A, B and S(x) this way from the moments and compares them
with the plain fine-grid products Z^T (K + M_W) Z, Z^T M Z and Z^T M_{(Zx)^2} Z built by
generic assembly on the fine mesh.  A dropped term or a wrong index in any moment (e.g. u~
in the place of a barycentric factor in T3) changes the matrices by O(1)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem
from oracle.mesh import Mesh


def _i4(d):
    """int_E l_i l_j l_k l_m / |E| from d! alpha! / (|alpha| + d)!, written out here."""
    nv = d + 1
    t = np.zeros((nv,) * 4)
    for idx in np.ndindex(*t.shape):
        alpha = [idx.count(v) for v in range(nv)]
        t[idx] = math.factorial(d) * math.prod(math.factorial(a) for a in alpha) / math.factorial(4 + d)
    return t


def _from_moments(c: Mesh, mo, KH, MH, x):
    d, N = c.dim, c.ndof
    I4 = _i4(d)
    A = np.zeros((N + 1, N + 1))
    B = np.zeros((N + 1, N + 1))
    S = np.zeros((N + 1, N + 1))
    A[:N, :N] = KH
    B[:N, :N] = MH
    cx = x[N]
    for E, el in enumerate(c.elems):
        ids = c.imap[el]
        X = np.array([x[a] if a >= 0 else 0.0 for a in ids])
        pts = c.coords[el]
        vol = abs(np.linalg.det(pts[1:] - pts[0])) / math.factorial(d)
        T3, T2, T1, T0 = mo["T3"][E], mo["T2"][E], mo["T1"][E], mo["T0"][E]
        Scc = vol * np.einsum("r,s,rspq->pq", X, X, I4) + 2 * cx * np.einsum("r,rpq->pq", X, T3) + cx ** 2 * T2
        Scu = np.einsum("r,s,rsp->p", X, X, T3) + 2 * cx * np.einsum("r,rp->p", X, T2) + cx ** 2 * T1
        Suu = X @ T2 @ X + 2 * cx * (X @ T1) + cx ** 2 * T0
        for p, a in enumerate(ids):
            if a < 0:
                continue
            B[a, N] += mo["B1"][E][p]
            A[a, N] += mo["KG"][E][p] + mo["AW1"][E][p]
            S[a, N] += Scu[p]
            for q, b in enumerate(ids):
                if b >= 0:
                    S[a, b] += Scc[p, q]
        B[N, N] += mo["B2"][E]
        A[N, N] += mo["Q"][E] + mo["AW2"][E]
        S[N, N] += Suu
    for Mx in (A, B, S):
        Mx[N, :N] = Mx[:N, N]
    return A, B, S


@pytest.mark.parametrize("dim, nc, refine", [(2, 4, 2), (3, 2, 2), (3, 3, 1)])
def test_moments_assemble_the_augmented_matrices(dim, nc, refine):
    rng = np.random.default_rng(7 + dim + nc)
    c, f = Mesh(dim, nc), Mesh(dim, nc << refine)
    W = fem.potential((0.7, 1.3, 1.9), 0.4)
    ut = rng.standard_normal(f.ndof)
    x = rng.standard_normal(c.ndof + 1)
    mo = fem.coarse_simplex_moments(c, f, ut, W)
    A, B, S = _from_moments(c, mo, (fem.stiffness(c) + fem.potential_mass(c, W)).toarray(), fem.mass(c).toarray(), x)
    Pi = fem.prolongation(f, c)
    Z = sp.hstack([Pi, sp.csr_matrix(ut[:, None])]).tocsr()
    A_ref = (Z.T @ ((fem.stiffness(f) + fem.potential_mass(f, W)) @ Z)).toarray()
    B_ref = (Z.T @ (fem.mass(f) @ Z)).toarray()
    S_ref = (Z.T @ (fem.density_mass(f, Z @ x) @ Z)).toarray()
    for got, want in ((A, A_ref), (B, B_ref), (S, S_ref)):
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_moments_of_a_coarse_function_are_coarse_integrals():
    """u~ = a coarse hat written on the fine mesh: every moment is an integral of products
    of barycentric coordinates over E, which the monomial formula gives in closed form."""
    c, f = Mesh(2, 3), Mesh(2, 12)
    a = 1   # an interior coarse dof
    e = np.zeros(c.ndof)
    e[a] = 1.0
    ut = fem.prolongation(f, c) @ e
    mo = fem.coarse_simplex_moments(c, f, ut)
    I4 = _i4(2)
    for E, el in enumerate(c.elems):
        ids = list(c.imap[el])
        vol = abs(np.linalg.det(c.coords[el][1:] - c.coords[el][0])) / 2
        if a not in ids:
            assert np.abs(mo["T3"][E]).max() == 0.0 and mo["T0"][E] == 0.0
            continue
        s = ids.index(a)
        # u~ = l_s on E
        assert np.allclose(mo["T3"][E], vol * I4[s], rtol=0, atol=1e-15)
        assert np.allclose(mo["T2"][E], vol * I4[s, s], rtol=0, atol=1e-15)
        assert np.allclose(mo["T1"][E], vol * I4[s, s, s], rtol=0, atol=1e-15)
        assert mo["T0"][E] == pytest.approx(vol * I4[s, s, s, s], rel=1e-13)
        assert mo["B2"][E] == pytest.approx(vol / 6.0, rel=1e-13)          # int l_s^2 = 2|E|/4!
