"""P1 finite-element assembly on simplex meshes (oracle side).

Section 2: the space V_h of continuous piecewise-linear functions vanishing on
the boundary (eq. "linear_fe_space"), the bilinear form a(u,v) = (grad u, grad v)
(the operator matrix A is the identity in every example of Section 4), and the
discrete problem eq. "FEM_form".

Quadrature reading: the L2 pairings (f(x,u), v) and (g, v) are taken with the
vertex (nodal) rule, (w, phi_j) ~ m_j w(x_j) with the lumped mass
m_j = sum_{T contains x_j} |T|/(d+1).  The paper writes exact integrals and
names no rule; the vertex rule keeps the P1 rates and positive weights, and is
used identically on every space, including the augmented space of
Algorithm 3.1.

Everything is assembled element by element from the vertex coordinates; no
stencil formula is used, so the stencil closed forms are independent checks.

Variable coefficient (the symmetric positive definite matrix A(x) of eq.
"semilinear equation"), read as constant on every cell of the mesh: the local
stiffness of a simplex T is |T| grad(lambda_i)^T A_T grad(lambda_j) with A_T
the matrix of the cell that contains T.  A coefficient array is either
kappa per cell (A = kappa I) or the d(d+1)/2 upper-triangle components per
cell, row by row (2D: a11, a12, a22; 3D: a11, a12, a13, a22, a23, a33), as an
array (components, cells); cells are numbered x fastest by lower corner.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def simplex_geometry(X: np.ndarray):
    """Barycentric-coordinate gradients and volumes of simplices.

    X: (E, d+1, d) vertex coordinates.  Returns (grads (E, d+1, d), vol (E,),
    C (E, d+1, d+1)) where lambda_i(x) = C[:,0,i] + x . C[:,1:,i].
    """
    E, dp1, d = X.shape
    M = np.concatenate([np.ones((E, dp1, 1)), X], axis=2)  # rows [1, x_v]
    C = np.linalg.inv(M)                                   # M @ C = I
    vol = np.abs(np.linalg.det(M)) / math.factorial(d)
    grads = np.transpose(C[:, 1:, :], (0, 2, 1))           # (E, d+1, d)
    return grads, vol, C


# Element loops are taken in chunks of this many simplices, so that the 3D
# 256^3 mesh (about 10^8 tetrahedra) fits in memory.  Meshes with fewer
# simplices are assembled in one chunk (the same operations as an unchunked
# loop); above it the duplicate entries of different chunks are added chunk by
# chunk, which only changes the order of rounding of those sums.
ELEMENT_CHUNK = 1 << 24


def cell_of_simplex(mesh: Mesh, T: np.ndarray) -> np.ndarray:
    """Index (x fastest) of the cell containing each simplex: the cell whose
    lower corner is the componentwise minimum of the simplex's vertices."""
    low = mesh.ijk[T].min(axis=1)                      # (E, d)
    idx = np.zeros(T.shape[0], dtype=np.int64)
    for a in range(mesh.dim - 1, -1, -1):
        idx = idx * mesh.n + low[:, a]
    return idx


def coefficient_tensors(dim: int, coef) -> np.ndarray:
    """(cells, d, d) symmetric matrices from a coefficient array (kappa per
    cell, or upper-triangle components per cell)."""
    c = np.asarray(coef, dtype=np.float64)
    if c.ndim == 1:
        return c[:, None, None] * np.eye(dim)[None]
    ncomp = dim * (dim + 1) // 2
    if c.shape[0] != ncomp:
        raise ValueError(f"expected {ncomp} components per cell, got {c.shape[0]}")
    out = np.empty((c.shape[1], dim, dim))
    q = 0
    for a in range(dim):
        for b in range(a, dim):
            out[:, a, b] = c[q]
            out[:, b, a] = c[q]
            q += 1
    return out


def _assemble_chunk(mesh: Mesh, T: np.ndarray, N: int, coef=None):
    X = mesh.coords[T]
    grads, vol, _ = simplex_geometry(X)
    d = mesh.dim
    if coef is None:
        Kloc = vol[:, None, None] * np.einsum("eia,eja->eij", grads, grads)
    else:
        At = coefficient_tensors(d, coef)[cell_of_simplex(mesh, T)]
        Kloc = vol[:, None, None] * np.einsum("eia,eab,ejb->eij", grads, At, grads)
    rows = np.repeat(T, d + 1, axis=1).reshape(-1)
    cols = np.tile(T, (1, d + 1)).reshape(-1)
    K = sp.csr_matrix((Kloc.reshape(-1), (rows, cols)), shape=(N, N))
    K.sum_duplicates()
    return K, vol


def assemble_full(mesh: Mesh, coef=None):
    """Full stiffness matrix (all nodes, CSR) and lumped mass vector.

    K_T[i,j] = |T| grad(lambda_i)^T A_T grad(lambda_j)  (local P1 stiffness;
    coef per cell as described above, or None for A = I).
    """
    d = mesh.dim
    N = mesh.coords.shape[0]
    mass = np.zeros(N)
    K = None
    for s in range(0, mesh.simplices.shape[0], ELEMENT_CHUNK):
        T = mesh.simplices[s:s + ELEMENT_CHUNK]
        Kc, vol = _assemble_chunk(mesh, T, N, coef)
        K = Kc if K is None else (K + Kc).tocsr()
        del Kc
        np.add.at(mass, T.reshape(-1), np.repeat(vol / (d + 1), d + 1))
    return K, mass


def assemble_interior(mesh: Mesh, coef=None):
    """Stiffness A (interior x interior, CSR) and lumped mass m on interior nodes.

    Dirichlet nodes are eliminated (u = 0 on the boundary, Section 2).
    """
    K, mass = assemble_full(mesh, coef)
    I = mesh.interior
    A = K[I][:, I].tocsr()
    A.sort_indices()
    return A, mass[I]


def simplices_around(dim: int, n: int, p: np.ndarray):
    """The simplices of the (0,1)^dim mesh with n cells per side that hold
    grid node p, generated from their definition: every cell whose closure
    holds p, split along every axis order into the vertex chain corner,
    corner + e_a0, ...  Yields (vertices (d+1, d) grid indices, cell corner)."""
    import itertools
    p = np.asarray(p, dtype=np.int64)
    for o in itertools.product((0, 1), repeat=dim):
        corner = p - np.array(o)
        if np.any(corner < 0) or np.any(corner >= n):
            continue
        for perm in itertools.permutations(range(dim)):
            v = [corner.copy()]
            for a in perm:
                w = v[-1].copy()
                w[a] += 1
                v.append(w)
            V = np.stack(v)
            if any(np.array_equal(x, p) for x in V):
                yield V, corner


def grid_node_id(n: int, ijk) -> int:
    """Node id (x fastest) of grid indices ijk on a mesh with n cells per side."""
    nid = 0
    for a in range(len(ijk) - 1, -1, -1):
        nid = nid * (n + 1) + int(ijk[a])
    return nid


def local_rows(dim: int, n: int, nodes_ijk: np.ndarray, coef=None):
    """Rows of the full stiffness matrix and lumped masses at a few nodes of
    the (0,1)^dim mesh with n cells per side, without building the mesh: the
    simplices around each node are generated from their definition (cells
    whose closure holds the node, split along every axis order into the chain
    of vertices corner, corner + e_a0, ..), and assembled with the same local
    formula as assemble_full.  Returns, per node, (column node ids x fastest,
    values) and the masses.  For checks at sizes whose full assembly does not
    fit in memory."""
    h = 1.0 / n
    nodes_ijk = np.asarray(nodes_ijk, dtype=np.int64)
    At = None if coef is None else coefficient_tensors(dim, coef)
    cols_out, vals_out, mass_out = [], [], []
    for p in nodes_ijk:
        row = {}
        mass = 0.0
        for V, corner in simplices_around(dim, n, p):
            X = V.astype(np.float64) * h
            grads, vol, _ = simplex_geometry(X[None])
            G = grads[0]
            if At is None:
                K = vol[0] * G @ G.T
            else:
                K = vol[0] * G @ At[_cell_index(n, corner)] @ G.T
            ip = next(k for k in range(dim + 1) if np.array_equal(V[k], p))
            for k in range(dim + 1):
                nid = grid_node_id(n, V[k])
                row[nid] = row.get(nid, 0.0) + K[ip, k]
            mass += vol[0] / (dim + 1)
        ids = np.array(sorted(row), dtype=np.int64)
        cols_out.append(ids)
        vals_out.append(np.array([row[i] for i in ids]))
        mass_out.append(mass)
    return cols_out, vals_out, np.array(mass_out)


def _cell_index(n: int, corner) -> int:
    """Cell id (x fastest) of the cell with lower corner `corner`."""
    cell = 0
    for a in range(len(corner) - 1, -1, -1):
        cell = cell * n + int(corner[a])
    return cell


def locate_in_coarse(coarse: Mesh, points: np.ndarray, tol: float = 1e-12):
    """Point location: for each point, a coarse simplex containing it and the
    point's barycentric coordinates in that simplex.

    The candidate simplices are those of the coarse cell floor(x n_c) (clamped),
    found through the cell's grid index; the containment test itself uses the
    generic barycentric coordinates of each candidate.
    """
    d, nc = coarse.dim, coarse.n
    cell = np.clip(np.floor(points * nc + 1e-9).astype(np.int64), 0, nc - 1)
    # map cell -> its simplices: simplices are stored as d! blocks of nc^d cells,
    # block p lists cells in 'ij' meshgrid order of (axis0, axis1, ...).
    ncell = nc ** d
    lin = np.zeros(points.shape[0], dtype=np.int64)
    for a in range(d):
        lin = lin * nc + cell[:, a]
    nperm = math.factorial(d)
    found_simplex = np.full(points.shape[0], -1, dtype=np.int64)
    found_bary = np.zeros((points.shape[0], d + 1))
    for p in range(nperm):
        sid = p * ncell + lin
        X = coarse.coords[coarse.simplices[sid]]
        _, _, C = simplex_geometry(X)
        bary = C[:, 0, :] + np.einsum("ea,eai->ei", points, C[:, 1:, :])
        ok = np.all(bary >= -tol, axis=1) & (found_simplex < 0)
        found_simplex[ok] = sid[ok]
        found_bary[ok] = bary[ok]
    if np.any(found_simplex < 0):
        raise RuntimeError("point location failed")
    return found_simplex, found_bary


def interpolation_matrix(coarse: Mesh, fine_points: np.ndarray) -> sp.csr_matrix:
    """Matrix evaluating coarse interior-node P1 functions at the given points.

    Entry (j, c) = phi_c(x_j): the natural inclusion V_coarse -> V_fine used by
    the nested spaces (eq. "FEM_Space_Series").  Columns are coarse interior
    nodes in ascending id order.
    """
    col_of = -np.ones(coarse.coords.shape[0], dtype=np.int64)
    col_of[coarse.interior] = np.arange(coarse.interior.size)
    vals, rows_all, cols_all = [], [], []
    # points are located independently, so taking them in chunks changes nothing
    for s in range(0, fine_points.shape[0], ELEMENT_CHUNK):
        pts = fine_points[s:s + ELEMENT_CHUNK]
        sid, bary = locate_in_coarse(coarse, pts)
        verts = coarse.simplices[sid]                   # (Nf, d+1) coarse node ids
        cols = col_of[verts]
        rows = np.repeat(np.arange(s, s + pts.shape[0]), coarse.dim + 1).reshape(cols.shape)
        keep = (cols >= 0) & (np.abs(bary) > 0)
        vals.append(bary[keep])
        rows_all.append(rows[keep])
        cols_all.append(cols[keep])
        del sid, bary, verts, cols, rows, keep
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows_all), np.concatenate(cols_all))),
                      shape=(fine_points.shape[0], coarse.interior.size))
    P.sum_duplicates()
    return P


def prolongation(coarse: Mesh, fine: Mesh) -> sp.csr_matrix:
    """P_k: V_{h_{k-1}} -> V_{h_k} on interior nodes (natural inclusion)."""
    return interpolation_matrix(coarse, fine.coords[fine.interior])
