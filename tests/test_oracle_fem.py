"""Pins for oracle.mesh and oracle.fem: element counts (Tables 1-2), the P1 forms of (2.2)
integrated exactly, and the nestedness (3.2) of the level spaces."""
import itertools
import math

import numpy as np
import pytest
import sympy as sp

from oracle import fem
from oracle.mesh import Mesh, interior_coords
from tests.symbolic import X, grid_simplices, integrate_simplex, p1_basis


# ---- meshes ----------------------------------------------------------------------------
@pytest.mark.parametrize("n, count", [(8, 3072), (16, 24576), (32, 196608)])
def test_3d_element_counts_match_table1(n, count):
    # Table 1 (and Table 2) list 3072, 24576, 196608, ... elements for h = 1/8, 1/16, ...
    assert Mesh(3, n).n_elements == count


def test_table1_counts_formula_for_larger_levels():
    # 6 n^3 continues the printed column: 1572864 (printed with a transposed digit) and 12582912.
    assert [6 * n ** 3 for n in (64, 128)] == [1572864, 12582912]


@pytest.mark.parametrize("dim, n, per_node", [(2, 6, 6), (3, 4, 24)])
def test_elements_per_interior_node(dim, n, per_node):
    m = Mesh(dim, n)
    counts = np.bincount(m.elems.ravel(), minlength=m.coords.shape[0])
    assert np.all(counts[m.imap >= 0] == per_node)
    assert m.n_elements == (2 if dim == 2 else 6) * n ** dim


@pytest.mark.parametrize("dim, n", [(2, 4), (3, 2)])
def test_regular_refinement_nests(dim, n):
    """Every fine simplex lies in one coarse simplex, which holds exactly 2^dim of them."""
    c, f = Mesh(dim, n), Mesh(dim, 2 * n)
    cx = c.coords[c.elems]
    T = np.concatenate([np.ones(cx.shape[:2] + (1,)), cx], axis=2)
    Cinv = np.linalg.inv(np.transpose(T, (0, 2, 1)))
    hits = np.zeros(c.n_elements, dtype=int)
    for el in f.elems:
        pts = f.coords[el]
        lam = np.einsum("eij,pj->epi", Cinv, np.concatenate([np.ones((dim + 1, 1)), pts], 1))
        inside = np.all(lam >= -1e-12, axis=(1, 2))
        assert inside.sum() == 1
        hits[np.argmax(inside)] += 1
    assert np.all(hits == 2 ** dim)


# ---- exact integration ----------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3])
def test_barycentric_monomial_identity_vs_sympy(d):
    rng = np.random.default_rng(1)
    verts = [tuple(sp.Rational(int(v), 5) for v in rng.integers(-5, 6, size=d)) for _ in range(d + 1)]
    lam = p1_basis(verts)
    vol = abs(integrate_simplex(sp.Integer(1), verts))
    assert vol != 0
    for alpha in [(1,) + (0,) * d, (2, 1) + (0,) * (d - 1), (1, 1, 1) + (0,) * (d - 2), (4,) + (0,) * d,
                  (0, 2, 0, 2)[: d + 1], (1, 1, 1, 1)[: d + 1]]:
        expr = sp.Mul(*[lam[i] ** a for i, a in enumerate(alpha)])
        exact = integrate_simplex(expr, verts) / vol
        assert float(exact) == pytest.approx(fem.bary_integral(alpha, d), rel=1e-14)


def test_power_integral_matches_complete_homogeneous_formula():
    """int_K u_h^p = |K| d! p!/(d+p)! h_p(u_0..u_d)  (h_p: complete homogeneous symmetric)."""
    m = Mesh(2, 3)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(m.ndof)
    uf = np.zeros(m.coords.shape[0]); uf[m.imap >= 0] = u
    for p in (2, 3, 4):
        tot = 0.0
        for el in m.elems:
            vals = uf[el]
            hp = sum(np.prod([vals[i] for i in c]) for c in itertools.combinations_with_replacement(range(3), p))
            tot += (0.5 / 9.0) * 2 * math.factorial(p) / math.factorial(2 + p) * hp
        assert fem.integral_of(m, u, p) == pytest.approx(tot, rel=1e-13)


def _sympy_global(dim, n, local):
    """Sum sympy element integrals local(verts, lam) -> dict[(a,b) or a] over the grid."""
    h = sp.Rational(1, n)
    out = {}
    for verts in grid_simplices(dim, n):
        lam = p1_basis(verts)
        idx = [tuple(int(sp.Integer(c / h)) for c in v) for v in verts]
        for key, val in local(verts, lam, idx).items():
            out[key] = out.get(key, 0) + val
    return out


def _dof(dim, n, ijk):
    if any(c in (0, n) for c in ijk):
        return -1
    i = [c - 1 for c in ijk]
    return i[0] + (n - 1) * (i[1] + ((n - 1) * i[2] if dim == 3 else 0))


@pytest.mark.parametrize("dim, n", [(2, 3), (3, 2)])
def test_potential_mass_and_cubic_load_vs_sympy(dim, n):
    """M_W and N(u) = int u^3 phi against symbolic integration of W phi_a phi_b and
    u_h^3 phi_a element by element, with W = 1.5 x^2 + 0.5 y^2 (+ 2 z^2) + 0.25."""
    wq = (1.5, 0.5, 2.0)[:dim]
    Wsym = sum(sp.Rational(str(w)) * X[k] ** 2 for k, w in enumerate(wq)) + sp.Rational(1, 4)
    m = Mesh(dim, n)
    rng = np.random.default_rng(3)
    u = np.array([sp.Rational(int(v), 7) for v in rng.integers(-7, 8, size=m.ndof)])
    u_num = u.astype(float)

    def local(verts, lam, idx):
        dofs = [_dof(dim, n, c) for c in idx]
        uh = sum(u[d] * lam[a] for a, d in enumerate(dofs) if d >= 0)
        out = {}
        for a, da in enumerate(dofs):
            if da < 0:
                continue
            out[("N", da)] = integrate_simplex(sp.expand(uh ** 3 * lam[a]), verts)
            for b, db in enumerate(dofs):
                if db >= 0:
                    out[(da, db)] = integrate_simplex(sp.expand(Wsym * lam[a] * lam[b]), verts)
        return out
    ref = _sympy_global(dim, n, local)
    MW = fem.potential_mass(m, fem.potential(wq, 0.25)).toarray()
    N = fem.nonlinear_load(m, u_num)
    for key, val in ref.items():
        if key[0] == "N":
            assert N[key[1]] == pytest.approx(float(val), rel=1e-13, abs=1e-16)
        else:
            assert MW[key] == pytest.approx(float(val), rel=1e-13, abs=1e-16)
    # density mass: u^T M_rho(u) u = int u^4 and M_rho(u) u = N(u)
    Mr = fem.density_mass(m, u_num)
    assert np.allclose(Mr @ u_num, N, rtol=1e-13, atol=1e-16)


# ---- stencils (closed forms derived by hand for these meshes) ---------------------------
def test_2d_stiffness_and_mass_stencils():
    n = 8
    m = Mesh(2, n)
    K = fem.stiffness(m).toarray()
    M = fem.mass(m).toarray()
    h2 = 1.0 / n ** 2
    i = 3 + 7 * 3                                  # node (4,4), dof (3,3)
    nb = {(1, 0): -1, (-1, 0): -1, (0, 1): -1, (0, -1): -1}
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            j = i + di + 7 * dj
            expect = 4.0 if (di, dj) == (0, 0) else nb.get((di, dj), 0.0)
            assert K[i, j] == pytest.approx(expect, abs=1e-14)
            mexp = 0.5 if (di, dj) == (0, 0) else (1 / 12 if (di, dj) in
                                                   [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)] else 0.0)
            assert M[i, j] == pytest.approx(mexp * h2, abs=1e-16)
    assert M[i].sum() == pytest.approx(h2, rel=1e-14)


def test_3d_stiffness_and_mass_stencils():
    n = 6
    m = Mesh(3, n)
    K = fem.stiffness(m).toarray()
    M = fem.mass(m).toarray()
    h = 1.0 / n
    s = n - 1
    i = 2 + s * (2 + s * 2)
    row_k = {}
    row_m = {}
    for dk, dj, di in itertools.product((-1, 0, 1), repeat=3):
        j = i + di + s * (dj + s * dk)
        row_k[(di, dj, dk)] = K[i, j]
        row_m[(di, dj, dk)] = M[i, j] / h ** 3
    for off, v in row_k.items():
        nz = sum(abs(c) for c in off)
        expect = 6 * h if nz == 0 else (-h if nz == 1 else 0.0)
        assert v == pytest.approx(expect, abs=1e-14)
    for off, v in row_m.items():
        if off == (0, 0, 0):
            e = 2 / 5
        elif sum(abs(c) for c in off) == 1 or off in [(1, 1, 1), (-1, -1, -1)]:
            e = 1 / 20
        elif off in [(1, 1, 0), (1, 0, 1), (0, 1, 1), (-1, -1, 0), (-1, 0, -1), (0, -1, -1)]:
            e = 1 / 30
        else:
            e = 0.0
        assert v == pytest.approx(e, abs=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_anisotropic_stiffness_couples_axis_neighbours_only(dim):
    """With A = diag(a): on these meshes only the axis-aligned edges carry a_d grad . grad
    (the edge directions of a right triangle / Kuhn tetrahedron along the path of axes), so
    the stiffness is the sum of a_d times the second-difference stencil along axis d:
    2D  [2 (a_x + a_y); -a_x on (+-1, 0), -a_y on (0, +-1)],
    3D  h [2 (a_x + a_y + a_z); -a_d on +-e_d].  Hand-derived closed form vs assembly."""
    n = 6
    a = (0.7, 1.9, 1.3)[:dim]
    m = Mesh(dim, n)
    K = fem.stiffness(m, a).toarray()
    s = n - 1
    scale = 1.0 if dim == 2 else 1.0 / n
    i = 2 + s * 2 + (s * s * 2 if dim == 3 else 0)
    for off in itertools.product((-1, 0, 1), repeat=dim):
        j = i + off[0] + s * off[1] + (s * s * off[2] if dim == 3 else 0)
        nz = [d for d in range(dim) if off[d] != 0]
        if not nz:
            expect = 2 * sum(a)
        elif len(nz) == 1:
            expect = -a[nz[0]]
        else:
            expect = 0.0
        assert K[i, j] == pytest.approx(expect * scale, abs=1e-14), off
    # A = I reproduces the isotropic matrix, and the form is linear in A
    assert abs(fem.stiffness(m, (1.0, 1.0, 1.0)) - fem.stiffness(m)).max() == 0.0
    b = (0.4, 0.8, 2.1)[:dim]
    Kab = fem.stiffness(m, tuple(x + y for x, y in zip(a, b)))
    assert abs(Kab - fem.stiffness(m, a) - fem.stiffness(m, b)).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_stiffness_on_quadratic_is_exact(dim):
    """K applied to the interpolant of x_k(1-x_k) equals int 2 phi_i (= 2 h^d) at every node."""
    n = 6 if dim == 3 else 10
    m = Mesh(dim, n)
    K = fem.stiffness(m)
    pts = interior_coords(dim, n)
    hat = fem.hat_integrals(m)
    h = 1.0 / n
    for k in range(dim):
        w = pts[:, k] * (1 - pts[:, k])
        # rows whose neighbours in the other directions are interior (w != 0 on those faces)
        rows = np.all([(pts[:, q] > 1.5 * h) & (pts[:, q] < 1 - 1.5 * h)
                       for q in range(dim) if q != k], axis=0)
        assert np.allclose((K @ w)[rows], 2 * hat[rows], rtol=1e-12, atol=1e-14)
    assert np.allclose(hat, (1.0 / n) ** dim)


# ---- transfer and Galerkin identities -------------------------------------------------------
def _hat_closed_form(pts, centre, H):
    """Hat function of these meshes: 1 - (max(0, X) - min(0, X)) over components, clipped."""
    X = (pts - centre) / H
    z = np.zeros((len(pts), 1))
    Xz = np.concatenate([X, z], axis=1)
    return np.maximum(0.0, 1.0 - (Xz.max(axis=1) - Xz.min(axis=1)))


@pytest.mark.parametrize("dim, nc, levels", [(2, 4, 3), (3, 2, 3)])
def test_composite_prolongation_is_coarse_hat(dim, nc, levels):
    from oracle.fmg import Hierarchy
    import workloads as W
    h = Hierarchy(W.Problem(dim, nc, levels - 1, (1, 1, 1), 0.0, 1.0))
    cpts = interior_coords(dim, nc)
    fpts = interior_coords(dim, nc << (levels - 1))
    Pi = h.Pi[-1].toarray()
    for c in range(len(cpts)):
        assert np.allclose(Pi[:, c], _hat_closed_form(fpts, cpts[c], 1.0 / nc), atol=1e-14)


@pytest.mark.parametrize("dim, nc", [(2, 4), (3, 2)])
def test_galerkin_identities(dim, nc):
    fine, coarse = Mesh(dim, 2 * nc), Mesh(dim, nc)
    P = fem.prolongation(fine, coarse)
    W = fem.potential((1.0, 2.0, 0.5), 0.3)
    for op in (fem.stiffness, fem.mass, lambda mm: fem.potential_mass(mm, W)):
        A_f, A_c = op(fine), op(coarse)
        assert abs(P.T @ A_f @ P - A_c).max() < 1e-13 * abs(A_c).max()
