"""Exact P1 finite-element integration on simplices (generic element loops).

Forms of the weak problem (2.2) and its discretisation (2.4):
  a-hat(w, v) = int A grad w . grad v                    (2.5), the stiffness matrix K; A = I
                                                          in the examples, a constant diagonal
                                                          SPD A = diag(a_1, .., a_d) in general
                                                          (the framework of Section 2 allows any
                                                          SPD coefficient)
  b(w, v)     = int w v                                   the mass matrix M
  int W w v                                               the potential part of f(x,u) (Example 4.1)
  int u^3 v                                               the cubic part of f(x,u) (Example 4.1, |u|^2 u = u^3)
The paper does not fix a quadrature (reading: every integrand is integrated exactly; W is a
quadratic polynomial, so all integrands are polynomials of degree <= 4 on each simplex).

Exact integration uses the barycentric-monomial identity on a d-simplex K:
    int_K lambda^alpha = d! |K| alpha! / (|alpha| + d)!
and a quadratic W is represented exactly by its P2 interpolant on each element.
Nothing here knows the stencils; everything is assembled element by element.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh

_CHUNK = 1 << 20


def bary_integral(alpha, d: int) -> float:
    """int_K prod lambda_i^alpha_i / |K|  =  d! alpha! / (|alpha| + d)!"""
    num = math.factorial(d)
    for a in alpha:
        num *= math.factorial(a)
    return num / math.factorial(sum(alpha) + d)


def bary_tensor(d: int, order: int) -> np.ndarray:
    """T[i1..ik] = int_K lambda_i1 ... lambda_ik / |K| for k = order."""
    nv = d + 1
    t = np.zeros((nv,) * order)
    for idx in itertools.product(range(nv), repeat=order):
        alpha = [idx.count(v) for v in range(nv)]
        t[idx] = bary_integral(alpha, d)
    return t


def element_geometry(coords: np.ndarray, elems: np.ndarray):
    """Volumes |K| (E,) and barycentric gradients (E, d+1, d) of the given elements."""
    x = coords[elems]                     # (E, d+1, d)
    d = x.shape[2]
    jac = x[:, 1:, :] - x[:, :1, :]       # rows: edge vectors
    det = np.linalg.det(jac)
    vol = np.abs(det) / math.factorial(d)
    # lambda = C @ [1, x]; C = inv(T^T), T rows = [1, x_j]
    T = np.concatenate([np.ones(x.shape[:2] + (1,)), x], axis=2)   # (E, d+1, d+1)
    C = np.linalg.inv(np.transpose(T, (0, 2, 1)))
    grads = C[:, :, 1:]
    return vol, grads


def potential(w_quad, w_const):
    """W(x) = sum_k w_k x_k^2 + c  (Example 4.1: all w_k = 1, c = 0)."""
    w = np.asarray(w_quad, dtype=np.float64)

    def W(x):
        return (x ** 2) @ w[: x.shape[-1]] + w_const
    return W


def _chunks(n):
    for s in range(0, n, _CHUNK):
        yield slice(s, min(n, s + _CHUNK))


def _assemble(mesh: Mesh, local_fn) -> sp.csr_matrix:
    """Sum element matrices local_fn(elem_slice) -> (E, d+1, d+1) into the interior block."""
    nv = mesh.dim + 1
    rows, cols, vals = [], [], []
    for sl in _chunks(mesh.n_elements):
        el = mesh.elems[sl]
        loc = local_fn(sl)
        r = np.repeat(el, nv, axis=1)
        c = np.tile(el, (1, nv))
        ri, ci = mesh.imap[r.ravel()], mesh.imap[c.ravel()]
        keep = (ri >= 0) & (ci >= 0)
        rows.append(ri[keep]); cols.append(ci[keep]); vals.append(loc.reshape(-1)[keep])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.ndof, mesh.ndof))
    return A.tocsr()


def _assemble_vec(mesh: Mesh, local_fn) -> np.ndarray:
    """Sum element vectors local_fn(elem_slice) -> (E, d+1) into the interior dofs."""
    out = np.zeros(mesh.ndof)
    for sl in _chunks(mesh.n_elements):
        el = mesh.elems[sl]
        loc = local_fn(sl)
        ii = mesh.imap[el.ravel()]
        keep = ii >= 0
        np.add.at(out, ii[keep], loc.ravel()[keep])
    return out


def stiffness(mesh: Mesh, diffusion=None) -> sp.csr_matrix:
    """K_ab = int A grad phi_a . grad phi_b  (a-hat of (2.5)); A = diag(diffusion), default I."""
    a = np.ones(mesh.dim) if diffusion is None else np.asarray(diffusion, dtype=float)[: mesh.dim]

    def loc(sl):
        vol, g = element_geometry(mesh.coords, mesh.elems[sl])
        return vol[:, None, None] * np.einsum("eak,k,ebk->eab", g, a, g)
    return _assemble(mesh, loc)


def mass(mesh: Mesh) -> sp.csr_matrix:
    """M_ab = int phi_a phi_b  (b of (2.2))."""
    I2 = bary_tensor(mesh.dim, 2)

    def loc(sl):
        vol, _ = element_geometry(mesh.coords, mesh.elems[sl])
        return vol[:, None, None] * I2[None]
    return _assemble(mesh, loc)


def _p2_values(mesh: Mesh, el: np.ndarray, W):
    """W at the vertices (E, d+1) and at the edge midpoints (E, d+1, d+1) of each element."""
    x = mesh.coords[el]
    wv = W(x)
    mid = 0.5 * (x[:, :, None, :] + x[:, None, :, :])
    return wv, W(mid)


def potential_mass(mesh: Mesh, W) -> sp.csr_matrix:
    """(M_W)_ab = int W phi_a phi_b, exact for quadratic W via its P2 interpolant
    W = sum_c W(v_c) lambda_c (2 lambda_c - 1) + sum_{c<e} 4 W(m_ce) lambda_c lambda_e."""
    d = mesh.dim
    I3, I4 = bary_tensor(d, 3), bary_tensor(d, 4)
    nv = d + 1

    def loc(sl):
        el = mesh.elems[sl]
        vol, _ = element_geometry(mesh.coords, el)
        wv, wm = _p2_values(mesh, el, W)
        out = np.einsum("ec,cab->eab", wv, 2.0 * np.einsum("ccab->cab", I4) - I3)
        for c in range(nv):
            for e in range(c + 1, nv):
                out += 4.0 * wm[:, c, e][:, None, None] * I4[c, e][None]
        return vol[:, None, None] * out
    return _assemble(mesh, loc)


def _full(mesh: Mesh, u: np.ndarray) -> np.ndarray:
    """Interior vector -> values at all grid nodes (zero Dirichlet ring)."""
    v = np.zeros(mesh.coords.shape[0])
    v[mesh.imap >= 0] = u
    return v


def nonlinear_load(mesh: Mesh, u: np.ndarray) -> np.ndarray:
    """N(u)_a = int u_h^3 phi_a  with u_h the P1 function of u."""
    I4 = bary_tensor(mesh.dim, 4)
    uf = _full(mesh, u)

    def loc(sl):
        el = mesh.elems[sl]
        vol, _ = element_geometry(mesh.coords, el)
        ue = uf[el]
        return vol[:, None] * np.einsum("ej,ek,el,jkla->ea", ue, ue, ue, I4)
    return _assemble_vec(mesh, loc)


def density_mass(mesh: Mesh, u: np.ndarray) -> sp.csr_matrix:
    """(M_rho)_ab = int u_h^2 phi_a phi_b  (the matrix of v -> u_h^2 v)."""
    I4 = bary_tensor(mesh.dim, 4)
    uf = _full(mesh, u)

    def loc(sl):
        el = mesh.elems[sl]
        vol, _ = element_geometry(mesh.coords, el)
        ue = uf[el]
        q = np.einsum("ej,ek->ejk", ue, ue).reshape(len(el), -1)
        return vol[:, None, None] * (q @ I4.reshape(-1, I4.shape[2] * I4.shape[3])).reshape(
            len(el), I4.shape[2], I4.shape[3])
    return _assemble(mesh, loc)


def integral_of(mesh: Mesh, u: np.ndarray, power: int = 1) -> float:
    """int u_h^power over the domain (exact)."""
    I = bary_tensor(mesh.dim, power)
    uf = _full(mesh, u)
    tot = 0.0
    for sl in _chunks(mesh.n_elements):
        el = mesh.elems[sl]
        vol, _ = element_geometry(mesh.coords, el)
        ue = uf[el]
        val = np.broadcast_to(I, (len(el),) + I.shape)
        for _ in range(power):
            val = np.einsum("ej,ej...->e...", ue, val)
        tot += float(vol @ val)
    return tot


def hat_integrals(mesh: Mesh) -> np.ndarray:
    """int phi_a for every interior dof."""
    def loc(sl):
        vol, _ = element_geometry(mesh.coords, mesh.elems[sl])
        return np.repeat(vol[:, None] / (mesh.dim + 1), mesh.dim + 1, axis=1)
    return _assemble_vec(mesh, loc)


def prolongation(fine: Mesh, coarse: Mesh) -> sp.csr_matrix:
    """P1 interpolation of coarse functions at the fine interior nodes (nestedness (3.2)).

    Generic point location: each fine node is located in a coarse simplex of its coarse
    cell and receives the coarse barycentric weights of that simplex's interior vertices."""
    d, nc = coarse.dim, coarse.n
    pts = fine.coords[fine.imap >= 0]
    cell = np.clip(np.floor(pts * nc + 1e-9).astype(np.int64), 0, nc - 1)
    lin = cell[:, 0] + nc * cell[:, 1] + (nc * nc * cell[:, 2] if d == 3 else 0)
    ncell = nc ** d
    ntype = coarse.n_elements // ncell
    rows, cols, vals = [], [], []
    done = np.zeros(len(pts), dtype=bool)
    for t in range(ntype):
        el = coarse.elems[t * ncell + lin]                 # candidate simplex per point
        x = coarse.coords[el]
        T = np.concatenate([np.ones(x.shape[:2] + (1,)), x], axis=2)
        lam = np.linalg.solve(np.transpose(T, (0, 2, 1)),
                              np.concatenate([np.ones((len(pts), 1)), pts], axis=1)[:, :, None])[:, :, 0]
        inside = (lam.min(axis=1) >= -1e-10) & ~done
        done |= inside
        idx = np.nonzero(inside)[0]
        for v in range(d + 1):
            cj = coarse.imap[el[idx, v]]
            w = lam[idx, v]
            keep = (cj >= 0) & (np.abs(w) > 1e-12)
            rows.append(idx[keep]); cols.append(cj[keep]); vals.append(w[keep])
    assert done.all(), "point location failed"
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.ndof, coarse.ndof)).tocsr()
    return P


def coarse_simplex_moments(coarse: Mesh, fine: Mesh, ut: np.ndarray, W=None):
    """Per coarse simplex E (in the coarse element order of mesh.simplices), the integrals
    of powers of the fine P1 function u~ against products of the barycentric coordinates
    l_p of E, all exact (products of P1 functions on each fine simplex):
        T3[pqr] = int_E u~ l_p l_q l_r,  T2[pq] = int_E u~^2 l_p l_q,  T1[p] = int_E u~^3 l_p,
        T0 = int_E u~^4,  B1[p] = int_E u~ l_p,  B2 = int_E u~^2,
        AW1[p] = int_E W u~ l_p, AW2 = int_E W u~^2 (when W is given),
        KG[p] = int_E grad u~ . grad l_p,  Q = int_E |grad u~|^2.
    Returns a dict of arrays indexed [E, ...].  Plain loops over fine simplices."""
    d = coarse.dim
    nv = d + 1
    I4 = bary_tensor(d, 4)
    uf = _full(fine, ut)
    cx = coarse.coords[coarse.elems]                        # (Ec, nv, d)
    Tc = np.concatenate([np.ones(cx.shape[:2] + (1,)), cx], axis=2)
    Cc = np.linalg.inv(np.transpose(Tc, (0, 2, 1)))          # lambda = Cc @ [1, x]
    fx = fine.coords[fine.elems]                             # (Ef, nv, d)
    cent = fx.mean(axis=1)
    # locate the coarse simplex of every fine simplex by its centroid
    lam_c = np.einsum("eij,fj->fei", Cc, np.concatenate([np.ones((len(cent), 1)), cent], 1))
    owner = np.argmax(np.all(lam_c >= -1e-12, axis=2), axis=1)
    assert np.all(np.all(lam_c[np.arange(len(cent)), owner] >= -1e-12, axis=1))
    vol, grads = element_geometry(fine.coords, fine.elems)
    out = {k: np.zeros((coarse.n_elements,) + sh) for k, sh in
           [("T3", (nv, nv, nv)), ("T2", (nv, nv)), ("T1", (nv,)), ("T0", ()), ("B1", (nv,)), ("B2", ()),
            ("AW1", (nv,)), ("AW2", ()), ("KG", (nv,)), ("Q", ())]}
    for f in range(fine.n_elements):
        E = owner[f]
        u = uf[fine.elems[f]]                                # values of u~ at the fine vertices
        pts = np.concatenate([np.ones((nv, 1)), fx[f]], 1)
        L = (Cc[E] @ pts.T).T                                # L[j, p] = l_p at fine vertex j
        v = vol[f]
        # int_e prod of four linear functions = v * I4 contracted with their vertex values
        one = np.ones(nv)
        out["T3"][E] += v * np.einsum("ijkl,i,jp,kq,lr->pqr", I4, u, L, L, L)
        out["T2"][E] += v * np.einsum("ijkl,i,j,kp,lq->pq", I4, u, u, L, L)
        out["T1"][E] += v * np.einsum("ijkl,i,j,k,lp->p", I4, u, u, u, L)
        out["T0"][E] += v * np.einsum("ijkl,i,j,k,l->", I4, u, u, u, u)
        out["B1"][E] += v * np.einsum("ijkl,i,jp,k,l->p", I4, u, L, one, one)
        out["B2"][E] += v * np.einsum("ijkl,i,j,k,l->", I4, u, u, one, one)
        gu = grads[f].T @ u                                   # gradient of u~ on e
        gl = np.linalg.inv(np.transpose(Tc[E]))[:, 1:]        # gradients of l_p
        out["KG"][E] += v * (gl @ gu)
        out["Q"][E] += v * (gu @ gu)
        if W is not None:
            # W is quadratic: exact through its P2 interpolant on e (as potential_mass)
            wv = W(fx[f])
            wm = W(0.5 * (fx[f][:, None, :] + fx[f][None, :, :]))
            I5 = bary_tensor(d, 5)
            I3 = bary_tensor(d, 3)
            # W u~ l_p and W u~^2 are degree <= 4; expand W = sum_c W_c l_c(2 l_c - 1) + sum 4 W_ce l_c l_e
            aw1 = np.zeros(nv)
            aw2 = 0.0
            for c in range(nv):
                e4 = 2.0 * np.einsum("ijkl,i,j,k,lp->p", I4, np.eye(nv)[c], np.eye(nv)[c], u, L) - \
                    np.einsum("ijk,i,j,kp->p", I3, np.eye(nv)[c], u, L)
                aw1 += wv[c] * e4
                aw2 += wv[c] * (2.0 * np.einsum("ijkl,i,j,k,l->", I4, np.eye(nv)[c], np.eye(nv)[c], u, u) -
                                np.einsum("ijk,i,j,k->", I3, np.eye(nv)[c], u, u))
                for e in range(c + 1, nv):
                    aw1 += 4.0 * wm[c, e] * np.einsum("ijkl,i,j,k,lp->p", I4, np.eye(nv)[c], np.eye(nv)[e], u, L)
                    aw2 += 4.0 * wm[c, e] * np.einsum("ijkl,i,j,k,l->", I4, np.eye(nv)[c], np.eye(nv)[e], u, u)
            out["AW1"][E] += v * aw1
            out["AW2"][E] += v * aw2
    return out
