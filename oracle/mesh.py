"""Nested uniform simplicial meshes of [0,1]^d and their P1 spaces.

Section 2 (the P1 space (2.3)) and Section 3 ((3.1) regular refinement with beta = 2 and
the nested spaces (3.2)).  The paper leaves the triangle orientation open (its initial-mesh
figure is not reproduced); the reading used here:
  * 2D: every cell [i,i+1]x[j,j+1] is cut by its (i,j)-(i+1,j+1) diagonal;
  * 3D: every cube is cut into the 6 Kuhn tetrahedra along its main diagonal, which gives
    the 6 n^3 element counts of Tables 1 and 2.
Both families reproduce themselves under one regular refinement.

Node numbering: grid node (i,j[,k]) has global index i + (n+1)(j + (n+1)k).
Interior (degree-of-freedom) numbering: (i-1) + (n-1)((j-1) + (n-1)(k-1)), x fastest.
"""
from __future__ import annotations

import itertools

import numpy as np


def grid_coords(dim: int, n: int) -> np.ndarray:
    """Coordinates of all (n+1)^dim grid nodes, x fastest."""
    t = np.arange(n + 1, dtype=np.float64) / n
    if dim == 2:
        y, x = np.meshgrid(t, t, indexing="ij")
        return np.stack([x.ravel(), y.ravel()], axis=1)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def _node(dim, n, idx):
    """Global node index from integer grid coordinates (arrays)."""
    g = n + 1
    if dim == 2:
        return idx[0] + g * idx[1]
    return idx[0] + g * (idx[1] + g * idx[2])


def simplices(dim: int, n: int) -> np.ndarray:
    """Element -> vertex table, shape (2n^2, 3) in 2D or (6n^3, 4) in 3D."""
    cells = np.stack(np.meshgrid(*([np.arange(n)] * dim), indexing="ij"), axis=-1)
    cells = cells.reshape(-1, dim)[:, ::-1]  # columns (i, j[, k]), x fastest
    out = []
    if dim == 2:
        corners = [[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]]
        for tri in corners:
            out.append(np.stack([_node(2, n, (cells[:, 0] + a, cells[:, 1] + b)) for a, b in tri],
                                axis=1))
    else:
        for perm in itertools.permutations(range(3)):
            verts = [np.zeros(3, dtype=int)]
            for ax in perm:
                v = verts[-1].copy()
                v[ax] += 1
                verts.append(v)
            out.append(np.stack([_node(3, n, (cells[:, 0] + v[0], cells[:, 1] + v[1],
                                              cells[:, 2] + v[2])) for v in verts], axis=1))
    return np.concatenate(out, axis=0).astype(np.int64)


def interior_map(dim: int, n: int) -> np.ndarray:
    """Array over global nodes: interior dof index, or -1 for boundary nodes."""
    g = n + 1
    idx = np.full(g ** dim, -1, dtype=np.int64)
    r = np.arange(1, n)
    if dim == 2:
        jj, ii = np.meshgrid(r, r, indexing="ij")
        idx[_node(2, n, (ii.ravel(), jj.ravel()))] = np.arange((n - 1) ** 2)
    else:
        kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
        idx[_node(3, n, (ii.ravel(), jj.ravel(), kk.ravel()))] = np.arange((n - 1) ** 3)
    return idx


def interior_coords(dim: int, n: int) -> np.ndarray:
    """Coordinates of the interior nodes in dof order."""
    c = grid_coords(dim, n)
    return c[interior_map(dim, n) >= 0]


def interior_parity(dim: int, n: int) -> np.ndarray:
    """(i + j [+ k]) mod 2 of every interior node in dof order (0 = red, 1 = black)."""
    r = np.arange(1, n)
    if dim == 2:
        jj, ii = np.meshgrid(r, r, indexing="ij")
        return ((ii + jj) % 2).ravel()
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    return ((ii + jj + kk) % 2).ravel()


class Mesh:
    """One uniform level: coordinates, elements, interior numbering."""

    def __init__(self, dim: int, n: int):
        self.dim, self.n = dim, n
        self.h = 1.0 / n
        self.coords = grid_coords(dim, n)
        self.elems = simplices(dim, n)
        self.imap = interior_map(dim, n)
        self.ndof = (n - 1) ** dim

    @property
    def n_elements(self) -> int:
        return self.elems.shape[0]
