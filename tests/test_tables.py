"""Pins for the constant tables the HIP kernels compile in (csrc/tables.h and
csrc/moment_tables.h), read from the header text and checked without the generators:

* the star mass moments add up to int phi_0 = 1 (unit lattice);
* the moment tables reproduce, for seeded integer corner values of a P1 function u on the
  unit cell, every integral int u^k Y^b (k = 1, 2 with |b| <= 4 - k) over the whole cell
  and over each of its simplices, and the cell integrals of grad u, as computed by exact
  iterated integration with sympy (no barycentric formula involved);
* the power-sum form the moment pass uses for the cubic and quartic terms (no table) gives
  the same integrals int u^3, int u^3 Y_d and int u^4 on every simplex."""
import itertools
import math
import os
import re

import numpy as np
import pytest
import sympy as sp

from tests.symbolic import X, integrate_simplex, p1_basis

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1502_04657_amd", "csrc")


def _array(name, header="tables.h"):
    text = open(os.path.join(CSRC, header)).read()
    m = re.search(r"%s((?:\[\d+\])+)\s*=\s*\{(.*?)\};" % re.escape(name), text, flags=re.S)
    assert m, name
    dims = [int(x) for x in re.findall(r"\[(\d+)\]", m.group(1))]
    vals = np.array([float(v) for v in re.findall(r"-?\d+(?:\.\d+)?(?:[eE][-+]?\d+)?", m.group(2))])
    return vals.reshape(dims)


def test_star_mass_moments_integrate_the_hat():
    for name in ("kM0_2D", "kM0_3D"):
        assert abs(_array(name).sum() - 1.0) < 1e-15


MON = {2: [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)],
       3: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1),
           (0, 0, 2), (3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 2, 1),
           (0, 1, 2), (0, 0, 3)]}


def _cell_simplices(D):
    if D == 2:
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


@pytest.mark.parametrize("D", [2, 3])
def test_moment_tables_are_exact(D):
    H = "moment_tables.h"
    rng = np.random.default_rng(11 + D)
    uc = [int(v) for v in rng.integers(-3, 4, size=1 << D)]
    simp = _cell_simplices(D)
    corner = _array(f"kCorner{D}D", H).astype(int)
    # the simplices of the table are those of the mesh description, in the same order
    for t, verts in enumerate(simp):
        assert [sum(c << i for i, c in enumerate(v)) for v in verts] == list(corner[t])
    nk = {1: len(MON[D]), 2: sum(1 for m in MON[D] if sum(m) <= 2), 3: D + 1}
    exact = {k: np.zeros(nk[k]) for k in (1, 2, 3)}
    quartic = []
    per_simplex = []
    grad = np.zeros(D)
    for t, verts in enumerate(simp):
        lam = p1_basis(verts)
        u = sum(uc[corner[t][v]] * lam[v] for v in range(D + 1))
        mine = {}
        for k in (1, 2, 3):
            mine[k] = np.array([float(integrate_simplex(u ** k * sp.Mul(*[X[d] ** m[d] for d in range(D)]), verts))
                                for m in MON[D][: nk[k]]])
            exact[k] += mine[k]
        per_simplex.append(mine)
        quartic.append(float(integrate_simplex(u ** 4, verts)))
        for d in range(D):
            grad[d] += float(integrate_simplex(sp.diff(u, X[d]), verts))
    # whole-cell tables, grouped by corner products
    C1, C2 = _array(f"kC1_{D}D", H), _array(f"kC2_{D}D", H)
    pairs = _array(f"kPair{D}D", H).astype(int)
    L1 = sum(uc[c] * C1[c] for c in range(1 << D))
    L2 = sum(uc[a] * uc[b] * C2[p] for p, (a, b) in enumerate(pairs))
    for got, k in ((L1, 1), (L2, 2)):
        assert np.allclose(got, exact[k], rtol=0, atol=1e-13), k
    CG = _array(f"kCG{D}D", H)
    assert np.allclose(sum(uc[c] * CG[c] for c in range(1 << D)), grad, rtol=0, atol=1e-14)
    # per-simplex tables: vertex multisets in lexicographic order
    E1, E2 = _array(f"kE1_{D}D", H), _array(f"kE2_{D}D", H)
    for t in range(len(simp)):
        uv = [uc[corner[t][v]] for v in range(D + 1)]
        l1 = sum(uv[v] * E1[t][v] for v in range(D + 1))
        l2 = sum(uv[a] * uv[b] * E2[t][i]
                 for i, (a, b) in enumerate(itertools.combinations_with_replacement(range(D + 1), 2)))
        for got, k in ((l1, 1), (l2, 2)):
            assert np.allclose(got, per_simplex[t][k], rtol=0, atol=1e-13), (t, k)
        # power sums p_k of the vertex values, h_k from them, unit cell (|t| D! = 1)
        p = [sum(v ** k for v in uv) for k in range(5)]
        h1, h2 = p[1], (p[1] ** 2 + p[2]) / 2
        h3 = (p[1] ** 3 + 3 * p[1] * p[2] + 2 * p[3]) / 6
        h4 = (p[1] ** 4 + 6 * p[1] ** 2 * p[2] + 3 * p[2] ** 2 + 8 * p[1] * p[3] + 6 * p[4]) / 24
        cubic = [math.factorial(3) / math.factorial(D + 3) * h3]
        bracket = [h3 + v * (h2 + v * (h1 + v)) for v in uv]
        for d in range(D):
            cubic.append(math.factorial(3) / math.factorial(D + 4) *
                         sum(bracket[v] for v in range(D + 1) if simp[t][v][d] == 1))
        assert np.allclose(cubic, per_simplex[t][3], rtol=0, atol=1e-13), t
        assert abs(math.factorial(4) / math.factorial(D + 4) * h4 - quartic[t]) < 1e-12, t
