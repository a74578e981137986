"""Derives the constant coefficient tables that the HIP kernels use and writes tables.h.

Run:  python paper_1502_04657_amd/csrc/gen_tables.py   (needs sympy; output is committed)

For both mesh families (2D: unit cells cut along the (0,0)-(1,1) diagonal; 3D: unit
cubes cut into the 6 Kuhn tetrahedra) and a node at the origin of the unit lattice, the
script integrates exactly over the elements of the node's star:
    m0[o]    = int phi_0 phi_o
    m1[k][o] = int x_k phi_0 phi_o
    m2[k][o] = int x_k^2 phi_0 phi_o
for every neighbour offset o.  On a mesh of spacing h, with the node at X, a quadratic
potential W = sum_k w_k x_k^2 + c gives the exact potential-mass row
    int W phi_i phi_j = h^d [ sum_k w_k (X_k^2 m0 + 2 X_k h m1[k] + h^2 m2[k]) + c m0 ],
and m0 h^d is the consistent mass stencil.  It also emits the exact degree-4 quadrature
rules used for the fine-grid moment integrals: on triangles two symmetric orbits
(a, a, 1-2a), (b, b, 1-2b) of 3 points each; on tetrahedra the centroid, the orbit
(a, a, a, 1-3a) (4 points) and the orbit (c, c, 1/2-c, 1/2-c) (6 points).  Parameters and
weights are the root of the moment equations of the symmetric polynomials up to degree 4
(solved to 40 digits and checked on every monomial).
"""
from __future__ import annotations

import itertools
import os

import sympy as sp

X = sp.symbols("x0:3")


def simplices(dim):
    """Elements of the unit-lattice mesh that touch the origin (all cells around it)."""
    out = []
    for cell in itertools.product((-1, 0), repeat=dim):
        if dim == 2:
            a = cell
            for tri in ([(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]):
                out.append([tuple(a[i] + v[i] for i in range(2)) for v in tri])
        else:
            for perm in itertools.permutations(range(3)):
                v = list(cell)
                verts = [tuple(v)]
                for ax in perm:
                    v = list(v)
                    v[ax] += 1
                    verts.append(tuple(v))
                out.append(verts)
    return [e for e in out if tuple([0] * dim) in e]


def bary(verts):
    d = len(verts) - 1
    T = sp.Matrix([[1] + list(v) for v in verts])
    C = T.T.inv()
    xs = sp.Matrix([1] + list(X[:d]))
    return [sp.expand((C[i, :] * xs)[0]) for i in range(d + 1)]


def integrate(expr, verts):
    d = len(verts) - 1
    V = [sp.Matrix(v) for v in verts]
    t = sp.symbols(f"t0:{d}")
    J = sp.Matrix.hstack(*[V[i + 1] - V[0] for i in range(d)])
    xt = V[0] + J * sp.Matrix(t)
    g = sp.expand(expr.subs({X[i]: xt[i] for i in range(d)}, simultaneous=True)) * abs(J.det())
    for k in reversed(range(d)):
        g = sp.integrate(g, (t[k], 0, 1 - sum(t[:k])))
    return sp.nsimplify(g)


def stencil(dim):
    zero = tuple([0] * dim)
    acc = {}
    for e in simplices(dim):
        lam = bary(e)
        a = e.index(zero)
        for b, vb in enumerate(e):
            o = vb
            ent = acc.setdefault(o, [0, [0] * dim, [0] * dim])
            ent[0] += integrate(lam[a] * lam[b], e)
            for k in range(dim):
                ent[1][k] += integrate(X[k] * lam[a] * lam[b], e)
                ent[2][k] += integrate(X[k] ** 2 * lam[a] * lam[b], e)
    offs = sorted(acc.keys(), key=lambda o: (sum(abs(c) for c in o), o))
    return offs, acc


def exact_simplex(f, lam, dim):
    """int over the unit simplex of the polynomial f(lambda) / volume (monomial identity)."""
    poly = sp.Poly(sp.expand(f), *lam)
    tot = 0
    for mon, cf in poly.terms():
        num = sp.factorial(dim)
        for a in mon:
            num *= sp.factorial(a)
        tot += cf * num / sp.factorial(sum(mon) + dim)
    return tot


def rule_2d():
    """6-point degree-4 rule on triangles: two orbits (t, t, 1-2t) with weights w (per
    point, relative to the area).  The four unknowns solve the moment equations of
    1, e2, e3, e2^2 (e_k: elementary symmetric polynomials of the barycentrics)."""
    lam = sp.symbols("l0:3")
    a, b, wa, wb = sp.symbols("a b wa wb")
    el = lambda k: sum(sp.Mul(*c) for c in itertools.combinations(lam, k))
    orbit = lambda t: [(t, t, 1 - 2 * t), (t, 1 - 2 * t, t), (1 - 2 * t, t, t)]
    eqs = []
    for f in (sp.Integer(1), el(2), el(3), el(2) ** 2):
        s = sum(wa * f.subs(dict(zip(lam, p))) for p in orbit(a)) + \
            sum(wb * f.subs(dict(zip(lam, p))) for p in orbit(b))
        eqs.append(sp.expand(s - exact_simplex(f, lam, 2)))
    ra, rb, rwa, rwb = sp.nsolve(eqs, [a, b, wa, wb], [0.4, 0.1, 1 / 6, 1 / 6], prec=40)
    assert 0 < rb < ra < 0.5 and rwa > 0 and rwb > 0
    pts = orbit(ra) + orbit(rb)
    wts = [rwa] * 3 + [rwb] * 3
    for mon in itertools.product(range(5), repeat=3):
        if sum(mon) > 4:
            continue
        f = sp.Mul(*[lam[i] ** mon[i] for i in range(3)])
        q = sum(w * f.subs(dict(zip(lam, p))) for w, p in zip(wts, pts))
        assert abs(q - exact_simplex(f, lam, 2)) < sp.Float(1e-30)
    return pts, wts


def rule_3d():
    """11-point degree-4 rule on tetrahedra: centroid (weight w0), orbit (a, a, a, 1-3a)
    (w1 per point), orbit (c, c, 1/2-c, 1/2-c) (w2 per point); the five unknowns solve the
    moment equations of 1, e2, e3, e4, e2^2.  (The centroid weight comes out negative; the
    rule integrates the polynomial integrands exactly all the same.)"""
    lam = sp.symbols("l0:4")
    a, c, w0, w1, w2 = sp.symbols("a c w0 w1 w2")
    el = lambda k: sum(sp.Mul(*cc) for cc in itertools.combinations(lam, k))
    q = sp.Rational(1, 4)
    s31 = lambda t: [tuple(1 - 3 * t if i == j else t for i in range(4)) for j in range(4)]
    s22 = lambda t: [tuple(t if i in pr else sp.Rational(1, 2) - t for i in range(4))
                     for pr in itertools.combinations(range(4), 2)]
    eqs = []
    for f in (sp.Integer(1), el(2), el(3), el(4), el(2) ** 2):
        sub = lambda p: f.subs(dict(zip(lam, p)))
        s = w0 * sub((q, q, q, q)) + sum(w1 * sub(p) for p in s31(a)) + sum(w2 * sub(p) for p in s22(c))
        eqs.append(sp.expand(s - exact_simplex(f, lam, 3)))
    ra, rc, rw0, rw1, rw2 = sp.nsolve(eqs, [a, c, w0, w1, w2], [0.1, 0.1, -0.05, 0.05, 0.1], prec=40)
    assert 0 < ra < sp.Rational(1, 4) and 0 < rc < sp.Rational(1, 2) and rw1 > 0 and rw2 > 0
    pts = [(q, q, q, q)] + s31(ra) + s22(rc)
    wts = [rw0] + [rw1] * 4 + [rw2] * 6
    for mon in itertools.product(range(5), repeat=4):
        if sum(mon) > 4:
            continue
        f = sp.Mul(*[lam[i] ** mon[i] for i in range(4)])
        val = sum(w * f.subs(dict(zip(lam, p))) for w, p in zip(wts, pts))
        assert abs(val - exact_simplex(f, lam, 3)) < sp.Float(1e-30)
    return pts, wts


def cell_elements(dim):
    """Sub-elements of the unit cell [0,1]^dim as vertex offsets from the cell corner."""
    if dim == 2:
        return [[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]]
    out = []
    for perm in itertools.permutations(range(3)):
        v = [0, 0, 0]
        verts = [tuple(v)]
        for ax in perm:
            v = list(v)
            v[ax] += 1
            verts.append(tuple(v))
        out.append(verts)
    return out


def node_star(dim):
    """Elements around a node, as the offsets of their other vertices (node = origin)."""
    zero = tuple([0] * dim)
    out = []
    for e in simplices(dim):
        out.append([v for v in e if v != zero])
    return out


def fmt(v):
    return f"{float(v):.17g}"


def main():
    out = ["// Generated by gen_tables.py -- exact values (the triangle rule: 40-digit roots) printed",
           "// to 17 significant digits.",
           "#pragma once", ""]
    for dim in (2, 3):
        offs, acc = stencil(dim)
        n = len(offs)
        out.append(f"// {dim}D star of a node: {n} offsets (lattice units), mass/potential moments")
        out.append(f"constexpr int kStencil{dim}D = {n};")
        out.append(f"static constexpr int kOff{dim}D[{n}][{dim}] = {{" +
                   ", ".join("{" + ", ".join(str(c) for c in o) + "}" for o in offs) + "};")
        out.append(f"static constexpr double kM0_{dim}D[{n}] = {{" +
                   ", ".join(fmt(acc[o][0]) for o in offs) + "};")
        out.append(f"static constexpr double kM1_{dim}D[{dim}][{n}] = {{" +
                   ", ".join("{" + ", ".join(fmt(acc[o][1][k]) for o in offs) + "}" for k in range(dim)) + "};")
        out.append(f"static constexpr double kM2_{dim}D[{dim}][{n}] = {{" +
                   ", ".join("{" + ", ".join(fmt(acc[o][2][k]) for o in offs) + "}" for k in range(dim)) + "};")
        out.append("")
    # element enumerations
    for dim in (2, 3):
        ce = cell_elements(dim)
        out.append(f"// {dim}D sub-elements of a unit cell: vertex offsets; barycentric lambda_p = a_p + g_p . X")
        out.append(f"constexpr int kCellElems{dim}D = {len(ce)};")
        out.append(f"static constexpr int kCellElemVert{dim}D[{len(ce)}][{dim + 1}][{dim}] = {{" +
                   ", ".join("{" + ", ".join("{" + ", ".join(str(c) for c in v) + "}" for v in e) + "}" for e in ce) + "};")
        coefs = []
        for e in ce:
            lam = bary(e)
            rows = []
            for l in lam:
                poly = sp.Poly(l, *X[:dim])
                rows.append([poly.coeff_monomial(1)] + [poly.coeff_monomial(X[k]) for k in range(dim)])
            coefs.append(rows)
        out.append(f"static constexpr double kCellElemBary{dim}D[{len(ce)}][{dim + 1}][{dim + 1}] = {{" +
                   ", ".join("{" + ", ".join("{" + ", ".join(fmt(c) for c in r) + "}" for r in e) + "}" for e in coefs) + "};")
        st = node_star(dim)
        out.append(f"// {dim}D elements around a node: offsets of the other {dim} vertices")
        out.append(f"constexpr int kStarElems{dim}D = {len(st)};")
        out.append(f"static constexpr int kStarElem{dim}D[{len(st)}][{dim}][{dim}] = {{" +
                   ", ".join("{" + ", ".join("{" + ", ".join(str(c) for c in v) + "}" for v in e) + "}" for e in st) + "};")
        out.append("")
    # quadrature rules
    pts, wts = rule_2d()
    out.append(f"// exact degree-4 rule on triangles: barycentric points, weights / area (sum 1)")
    out.append(f"constexpr int kQuad2D = {len(pts)};")
    out.append("static constexpr double kQuadPt2D[%d][3] = {%s};" % (
        len(pts), ", ".join("{" + ", ".join(fmt(c) for c in p) + "}" for p in pts)))
    out.append("static constexpr double kQuadW2D[%d] = {%s};" % (len(pts), ", ".join(fmt(w) for w in wts)))
    pts, wts = rule_3d()
    out.append(f"// exact degree-4 rule on tetrahedra: barycentric points, weights / volume (sum 1)")
    out.append(f"constexpr int kQuad3D = {len(pts)};")
    out.append("static constexpr double kQuadPt3D[%d][4] = {%s};" % (
        len(pts), ", ".join("{" + ", ".join(fmt(c) for c in p) + "}" for p in pts)))
    out.append("static constexpr double kQuadW3D[%d] = {%s};" % (len(pts), ", ".join(fmt(w) for w in wts)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables.h")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
