"""Exact symbolic integration over simplices (sympy), used to pin the oracle.

Independent of the oracle: integrals are taken by iterated integration of polynomials
over the simplex, with no barycentric formula involved."""
from __future__ import annotations

import itertools

import sympy as sp

X = sp.symbols("x0:3")


def integrate_simplex(expr, verts):
    """int over the simplex with the given vertices (list of d+1 points) of a polynomial
    in x0..x{d-1}, by the affine map from the unit simplex and iterated integration."""
    d = len(verts) - 1
    V = [sp.Matrix([sp.nsimplify(c) for c in v]) for v in verts]
    t = sp.symbols(f"t0:{d}")
    J = sp.Matrix.hstack(*[V[i + 1] - V[0] for i in range(d)])
    x_of_t = V[0] + J * sp.Matrix(t)
    g = sp.expand(expr.subs({X[i]: x_of_t[i] for i in range(d)}, simultaneous=True)) * abs(J.det())
    # unit simplex: t_i >= 0, sum t_i <= 1; integrate t_{d-1} first.
    for k in reversed(range(d)):
        upper = 1 - sum(t[:k])
        g = sp.integrate(g, (t[k], 0, upper))
    return sp.nsimplify(g)


def p1_basis(verts):
    """Barycentric coordinates of the simplex as sympy polynomials in x0..x{d-1}."""
    d = len(verts) - 1
    T = sp.Matrix([[1] + [sp.nsimplify(c) for c in v] for v in verts])   # rows [1, x_j]
    C = T.T.inv()
    xs = sp.Matrix([1] + list(X[:d]))
    return [sp.expand((C[i, :] * xs)[0]) for i in range(d + 1)]


def grid_simplices(dim, n):
    """The mesh of [0,1]^dim, written out independently of the oracle's mesh module:
    2D cells cut along the (i,j)-(i+1,j+1) diagonal, 3D cubes cut into 6 Kuhn tetrahedra."""
    out = []
    h = sp.Rational(1, n)
    for cell in itertools.product(range(n), repeat=dim):
        base = [c * h for c in cell]
        if dim == 2:
            a = (base[0], base[1])
            out.append([a, (a[0] + h, a[1]), (a[0] + h, a[1] + h)])
            out.append([a, (a[0] + h, a[1] + h), (a[0], a[1] + h)])
        else:
            for perm in itertools.permutations(range(3)):
                v = list(base)
                verts = [tuple(v)]
                for ax in perm:
                    v = list(v)
                    v[ax] += h
                    verts.append(tuple(v))
                out.append(verts)
    return out
