"""Structured simplex meshes of the unit square / cube (oracle side).

Section 2 (shape-regular triangulations) and Section 3 (eq. "mesh_size_recur":
each refinement halves h and produces beta^d children).  The unit cube is cut
into n^d cells; every cell is split into d! simplices that all contain the
cell's main diagonal (Kuhn / Freudenthal split; in 2D the diagonal from
(0,0) to (1,1)).  Refining this mesh once (edge midpoints) gives the same kind
of mesh with n doubled, so the spaces are nested (eq. "FEM_Space_Series").

Node numbering: index = i_x + (n+1) i_y (+ (n+1)^2 i_z), x fastest.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    dim: int
    n: int                      # cells per side
    coords: np.ndarray          # (N, d) node coordinates
    ijk: np.ndarray             # (N, d) integer grid indices (x first)
    simplices: np.ndarray       # (E, d+1) node ids
    boundary: np.ndarray        # (N,) bool
    interior: np.ndarray        # (N_int,) node ids of interior nodes, ascending

    @property
    def h(self) -> float:
        return 1.0 / self.n


def node_id(ijk: np.ndarray, n: int) -> np.ndarray:
    d = ijk.shape[-1]
    out = np.zeros(ijk.shape[:-1], dtype=np.int64)
    for a in range(d - 1, -1, -1):
        out = out * (n + 1) + ijk[..., a]
    return out


def unit_mesh(dim: int, n: int) -> Mesh:
    """(0,1)^dim cut into n^dim cells and d! simplices per cell."""
    N = (n + 1) ** dim
    ids = np.arange(N, dtype=np.int64)
    ijk = np.empty((N, dim), dtype=np.int64)
    rem = ids.copy()
    for a in range(dim):
        ijk[:, a] = rem % (n + 1)
        rem //= (n + 1)
    coords = ijk.astype(np.float64) / n
    boundary = np.any((ijk == 0) | (ijk == n), axis=1)

    # cells by lower corner
    corners = np.stack(np.meshgrid(*([np.arange(n)] * dim), indexing="ij"), -1).reshape(-1, dim)
    simp = []
    for perm in itertools.permutations(range(dim)):
        verts = [corners.copy()]
        cur = corners.copy()
        for axis in perm:
            cur = cur.copy()
            cur[:, axis] += 1
            verts.append(cur)
        simp.append(np.stack([node_id(v, n) for v in verts], axis=1))
    simplices = np.concatenate(simp, axis=0)
    return Mesh(dim, n, coords, ijk, simplices, boundary, np.nonzero(~boundary)[0])
