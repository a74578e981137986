"""Writes linear_eigs.json: the lowest eigenvalue of the discrete linear problem (zeta = 0,
W = 0) of (2.4), i.e. of the pencil (K, M) on the interior nodes, for a few uniform meshes.

Independent of oracle/ and of the HIP library: K and M are written here from their
closed-form stencils on the two mesh families (2D: cells cut along the (i,j)-(i+1,j+1)
diagonal; 3D: 6 Kuhn tetrahedra per cube),
    2D  K = [4; -1 on (+-1,0), (0,+-1)],  M = h^2 [1/2; 1/12 on (+-1,0), (0,+-1), +-(1,1)]
    3D  K = h [6; -1 on +-e_i],           M = h^3 [2/5; 1/20 on +-e_i and +-(1,1,1);
                                                   1/30 on +-(e_i + e_j)],
and the eigenvalue comes from scipy's shift-invert Lanczos.  For the continuous problem the
values are 2 pi^2 (2D) and 3 pi^2 (3D); P1 elements approach them from above at O(h^2).

    python tests/golden/make_linear_eigs.py
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [(2, 8), (2, 16), (2, 32), (2, 64), (3, 4), (3, 8), (3, 16)]


def stencil_matrix(dim, n, entries):
    """Sparse matrix on the (n-1)^dim interior nodes (x fastest) from {offset: weight}."""
    m = n - 1
    idx = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]
    lin = lambda c: sum(c[:, a] * m ** a for a in range(dim))   # noqa: E731
    rows, cols, vals = [], [], []
    for off, w in entries.items():
        nb = idx + np.asarray(off)
        ok = np.all((nb >= 0) & (nb < m), axis=1)
        rows.append(lin(idx[ok])); cols.append(lin(nb[ok])); vals.append(np.full(ok.sum(), w))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m ** dim,) * 2)


def pencil(dim, n):
    h = 1.0 / n
    units = [tuple(int(a == b) for b in range(dim)) for a in range(dim)]
    neg = lambda o: tuple(-v for v in o)   # noqa: E731
    K = {(0,) * dim: 2.0 * dim}
    for e in units:
        K[e] = K[neg(e)] = -1.0
    if dim == 2:
        M = {(0, 0): 0.5}
        for o in units + [(1, 1)]:
            M[o] = M[neg(o)] = 1.0 / 12.0
        return stencil_matrix(2, n, K), stencil_matrix(2, n, M) * h * h
    M = {(0, 0, 0): 0.4}
    for o in units + [(1, 1, 1)]:
        M[o] = M[neg(o)] = 1.0 / 20.0
    for a, b in itertools.combinations(range(3), 2):
        o = tuple(int(c in (a, b)) for c in range(3))
        M[o] = M[neg(o)] = 1.0 / 30.0
    return stencil_matrix(3, n, K) * h, stencil_matrix(3, n, M) * h ** 3


def lowest(dim, n):
    K, M = pencil(dim, n)
    w = sla.eigsh(K.tocsc(), k=1, M=M.tocsc(), sigma=0.0, which="LM", tol=1e-14)[0]
    return float(w[0])


if __name__ == "__main__":
    out = {"description": "lowest eigenvalue of (K, M), zeta = 0, W = 0, P1 on uniform meshes",
           "values": [{"dim": d, "n": n, "lambda": lowest(d, n)} for d, n in CASES]}
    with open(os.path.join(HERE, "linear_eigs.json"), "w") as f:
        json.dump(out, f, indent=1)
    for v in out["values"]:
        print(v)
