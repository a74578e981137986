"""Derives the exact coefficient tables of the fine-grid moment pass and writes
moment_tables.h.

Run:  python paper_1502_04657_amd/csrc/gen_moment_tables.py   (standard library only;
      the output is committed)

The moment pass integrates powers of a fine P1 function u~ against monomials of the
coordinates over the fine simplices of one unit cell (2D: the two triangles of a square
cut along its (0,0)-(1,1) diagonal; 3D: the six Kuhn tetrahedra of a cube, vertex order as
in tables.h).  On a simplex with barycentric coordinates l_v and vertex values u_v,
u~ = sum_v u_v l_v and every cell coordinate Y_d = sum_v y_vd l_v is linear, so

    int u~^k Y^b = sum over multisets {v_1..v_k} of vertices of (multinomial) u_v1..u_vk
                   * int l_v1 .. l_vk Y^b,

and int l^alpha = D! |simplex| alpha! / (|alpha| + D)! (the barycentric monomial
formula) gives every coefficient as an exact rational.  Emitted (cell-local coordinates Y,
unit cell, so the cell measure is 1):

  per simplex type t (vertex multisets in lexicographic order):
    E1[t][v][q]   = int_t l_v Y^{m_q}                        |m_q| <= 3
    E2[t][vw][q]  = mult(v,w) int_t l_v l_w Y^{m_q}          |m_q| <= 2
  for the whole cell, grouped by cell corners c (c = o_0 + 2 o_1 (+ 4 o_2)):
    C1[c][q], C2[pair][q]: the sums of the above over the cell's simplices with the same
    corner multiset (pairs that share a simplex),
    CG[c][d] = sum_t |t| d l_{v(c)} / dY_d,
with the monomial orders of layout.h (graded: degree 0, 1, 2, 3).  The cubic and quartic
terms need no table: with h_k the complete homogeneous symmetric polynomials of the
vertex values, int_t u~^k = |t| D! k! / (D+k)! h_k and
int_t u~^3 l_w = |t| D! 3! / (D+4)! (h_3 + u_w h_2 + u_w^2 h_1 + u_w^3).
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))

VERT = {
    2: [[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]],
    3: [[(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)], [(0, 0, 0), (1, 0, 0), (1, 0, 1), (1, 1, 1)],
        [(0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 1, 1)], [(0, 0, 0), (0, 1, 0), (0, 1, 1), (1, 1, 1)],
        [(0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1)], [(0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1)]],
}
MON = {
    2: [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)],
    3: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1),
        (0, 0, 2), (3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 2, 1),
        (0, 1, 2), (0, 0, 3)],
}


def corner(o):
    return sum(v << i for i, v in enumerate(o))


def poly_mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return out


def simplex_integral(poly, D):
    """int over a unit-cell simplex (measure 1/D!) of a polynomial in the l_v."""
    tot = Fraction(0)
    for alpha, c in poly.items():
        num = math.factorial(D) * math.prod(math.factorial(a) for a in alpha)
        tot += c * Fraction(num, math.factorial(sum(alpha) + D)) / math.factorial(D)
    return tot


def lam(v, D):
    e = [0] * (D + 1)
    e[v] = 1
    return {tuple(e): Fraction(1)}


def coord_power(verts, mono, D):
    """Y^mono as a polynomial in the barycentric coordinates of the simplex."""
    p = {tuple([0] * (D + 1)): Fraction(1)}
    for d, e in enumerate(mono):
        yd = {}
        for v, x in enumerate(verts):
            if x[d]:
                k = [0] * (D + 1)
                k[v] = 1
                yd[tuple(k)] = Fraction(1)
        for _ in range(e):
            p = poly_mul(p, yd)
    return p


def multiplicity(ms):
    return Fraction(math.factorial(len(ms)), math.prod(math.factorial(ms.count(x)) for x in set(ms)))


def tables(D):
    NS = len(VERT[D])
    deg_count = {1: len(MON[D]), 2: sum(1 for m in MON[D] if sum(m) <= 2)}
    E = {k: [] for k in (1, 2)}
    cells = {k: {} for k in (1, 2)}
    for t, verts in enumerate(VERT[D]):
        for k in (1, 2):
            rows = []
            for ms in itertools.combinations_with_replacement(range(D + 1), k):
                lp = {tuple([0] * (D + 1)): Fraction(1)}
                for v in ms:
                    lp = poly_mul(lp, lam(v, D))
                row = [multiplicity(list(ms)) * simplex_integral(poly_mul(lp, coord_power(verts, MON[D][q], D)), D)
                       for q in range(deg_count[k])]
                rows.append(row)
                key = tuple(sorted(corner(verts[v]) for v in ms))
                acc = cells[k].setdefault(key, [Fraction(0)] * deg_count[k])
                for q in range(deg_count[k]):
                    acc[q] += row[q]
            E[k].append(rows)
    # cell gradients: sum_t |t| grad l_v, grouped by corner
    CG = {c: [Fraction(0)] * D for c in range(1 << D)}
    for verts in VERT[D]:
        # l_v = a_v + g_v . Y from the vertex coordinates
        import fractions  # noqa: F401
        M = [[Fraction(1)] + [Fraction(x) for x in v] for v in verts]   # rows: [1, y_v]
        inv = mat_inv([list(r) for r in zip(*M)])                       # columns -> coefficients
        for v, x in enumerate(verts):
            for d in range(D):
                CG[corner(x)][d] += inv[v][1 + d] / math.factorial(D)
    return E, cells, CG


def mat_inv(A):
    n = len(A)
    M = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def fmt(x):
    return repr(float(x))


def arr(name, data, ctype="double"):
    def rec(d):
        if isinstance(d, list):
            return "{" + ", ".join(rec(x) for x in d) + "}"
        return fmt(d) if ctype == "double" else str(d)
    dims = []
    d = data
    while isinstance(d, list):
        dims.append(len(d))
        d = d[0]
    return f"static constexpr {ctype} {name}" + "".join(f"[{n}]" for n in dims) + " = " + rec(data) + ";"


def main():
    out = ["// Generated by gen_moment_tables.py -- exact rationals printed as doubles (17 digits).",
           "#pragma once", ""]
    for D in (2, 3):
        E, cells, CG = tables(D)
        nc = 1 << D
        pairs = sorted(cells[2])
        out.append(f"// ---- {D}D: cell corners c = o0 + 2 o1" + (" + 4 o2" if D == 3 else ""))
        out.append(arr(f"kCorner{D}D", [[corner(v) for v in verts] for verts in VERT[D]], "int"))
        out.append(f"constexpr int kPairs{D}D = {len(pairs)};")
        out.append(arr(f"kPair{D}D", [list(p) for p in pairs], "int"))
        out.append(arr(f"kC1_{D}D", [cells[1][(c,)] for c in range(nc)]))
        out.append(arr(f"kC2_{D}D", [cells[2][p] for p in pairs]))
        out.append(arr(f"kCG{D}D", [CG[c] for c in range(nc)]))
        out.append(arr(f"kE1_{D}D", E[1]))
        out.append(arr(f"kE2_{D}D", E[2]))
        out.append("")
    with open(os.path.join(HERE, "moment_tables.h"), "w") as f:
        f.write("\n".join(out))
    print("wrote moment_tables.h")


if __name__ == "__main__":
    main()
