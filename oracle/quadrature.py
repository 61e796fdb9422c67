"""Element quadrature of the L2 pairings (oracle side; test infrastructure).

The discrete problem of Section 2 (eq. "FEM_form") and the augmented problem
of Algorithm 3.1 (eq. "coarse problem") contain the exact integrals
(f(x, u_h), v_h) and (g, v_h).  The default reading replaces them by the
vertex rule (oracle/fem.py); this module is the element reading: on every
simplex T the integrand is evaluated at the points of a symmetric rule that
is exact for polynomials of degree 2 and weighted with |T|,

    (w, v)_T ~ |T| sum_q omega_q w(x_q) v(x_q),

with u_h, v_h and the load g taken as their P1 interpolants (so g enters
through its nodal values, and (g_I, v_h) is the consistent-mass product).
Rules (barycentric points, weights summing to 1):
  * triangles: the three points with coordinates (2/3, 1/6, 1/6) and
    permutations, weight 1/3 each;
  * tetrahedra: the four points (a, b, b, b) and permutations,
    a = (5 + 3 sqrt 5) / 20, b = (5 - sqrt 5) / 20, weight 1/4 each.

Every function works on nodal vectors over all mesh nodes (boundary values
included; u_h vanishes there) and returns vectors or matrices over all nodes;
callers restrict to interior nodes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .fem import ELEMENT_CHUNK, grid_node_id, simplex_geometry, simplices_around
from .mesh import Mesh
from .nonlinear import Nonlinearity


def simplex_rule(d: int):
    """(points (Q, d+1) barycentric, weights (Q,)) of the degree-2 rule."""
    if d == 2:
        a, b = 2.0 / 3.0, 1.0 / 6.0
        pts = np.array([[a, b, b], [b, a, b], [b, b, a]])
        return pts, np.full(3, 1.0 / 3.0)
    if d == 3:
        s5 = math.sqrt(5.0)
        a, b = (5.0 + 3.0 * s5) / 20.0, (5.0 - s5) / 20.0
        pts = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
        return pts, np.full(4, 0.25)
    raise ValueError(d)


class ElementQuadrature:
    """The degree-2 element rule on every simplex of one mesh."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        self.N = mesh.coords.shape[0]
        self.T = mesh.simplices
        vols = []
        for s in range(0, self.T.shape[0], ELEMENT_CHUNK):
            _, vol, _ = simplex_geometry(mesh.coords[self.T[s:s + ELEMENT_CHUNK]])
            vols.append(vol)
        self.vol = np.concatenate(vols)
        self.lam, self.omega = simplex_rule(mesh.dim)

    def _at_points(self, v: np.ndarray) -> np.ndarray:
        """Values of the P1 interpolant of nodal v at every quadrature point: (E, Q)."""
        return v[self.T] @ self.lam.T

    def _scatter(self, wq: np.ndarray) -> np.ndarray:
        """sum over simplices and points of |T| omega_q wq[e, q] lambda_{q,i} into node i."""
        contrib = (self.vol[:, None] * wq * self.omega[None, :]) @ self.lam   # (E, d+1)
        out = np.zeros(self.N)
        np.add.at(out, self.T.reshape(-1), contrib.reshape(-1))
        return out

    def load(self, g_nodes: np.ndarray) -> np.ndarray:
        """(g_I, phi_i) for every node i."""
        return self._scatter(self._at_points(np.asarray(g_nodes, dtype=np.float64)))

    def nonlinear(self, u_nodes: np.ndarray, nl: Nonlinearity) -> np.ndarray:
        """(f(u_h), phi_i) for every node i."""
        return self._scatter(nl.f(self._at_points(u_nodes)))

    def energy(self, u_nodes: np.ndarray, nl: Nonlinearity) -> float:
        """(F(u_h), 1): the quadrature of the antiderivative (F' = f)."""
        Fq = nl.F(self._at_points(u_nodes))
        return float(np.sum(self.vol * (Fq @ self.omega)))

    def weighted_mass(self, wq: np.ndarray) -> sp.csr_matrix:
        """Matrix sum_T |T| sum_q omega_q wq[e, q] lambda_{q,i} lambda_{q,j}."""
        d1 = self.T.shape[1]
        loc = np.einsum("eq,q,qi,qj->eij", self.vol[:, None] * wq, self.omega, self.lam, self.lam)
        rows = np.repeat(self.T, d1, axis=1).reshape(-1)
        cols = np.tile(self.T, (1, d1)).reshape(-1)
        K = sp.csr_matrix((loc.reshape(-1), (rows, cols)), shape=(self.N, self.N))
        K.sum_duplicates()
        return K

    def jacobian(self, u_nodes: np.ndarray, nl: Nonlinearity) -> sp.csr_matrix:
        """Derivative of nonlinear(u) in u: the f'(u_h)-weighted mass matrix."""
        return self.weighted_mass(nl.df(self._at_points(u_nodes)))


def full_vector(mesh: Mesh, U_interior: np.ndarray) -> np.ndarray:
    """Nodal values on all nodes from interior values (zero on the boundary)."""
    out = np.zeros(mesh.coords.shape[0])
    out[mesh.interior] = U_interior
    return out


def local_element_terms(dim: int, n: int, nodes_ijk, u_nodes: np.ndarray, g_nodes: np.ndarray, nl: Nonlinearity):
    """(f(u_h), phi_i) and (g_I, phi_i) at a few grid nodes i of the (0,1)^dim
    mesh with n cells per side, by the element rule on the simplices around
    each node only (fem.simplices_around): the same per-simplex formula as
    ElementQuadrature, for sizes whose whole mesh does not fit in memory."""
    lam, omega = simplex_rule(dim)
    h = 1.0 / n
    N, G = [], []
    for p in np.asarray(nodes_ijk, dtype=np.int64):
        nv = gv = 0.0
        for V, _ in simplices_around(dim, n, p):
            _, vol, _ = simplex_geometry((V.astype(np.float64) * h)[None])
            ids = [grid_node_id(n, v) for v in V]
            ip = next(k for k in range(dim + 1) if np.array_equal(V[k], p))
            uq = lam @ np.asarray(u_nodes)[ids]
            gq = lam @ np.asarray(g_nodes)[ids]
            nv += vol[0] * np.sum(omega * nl.f(uq) * lam[:, ip])
            gv += vol[0] * np.sum(omega * gq * lam[:, ip])
        N.append(nv)
        G.append(gv)
    return np.array(N), np.array(G)
