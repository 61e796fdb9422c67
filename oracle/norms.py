"""Error norms (oracle side).

* Nodal L2 norm ||v|| = (sum_j m_j v_j^2)^{1/2} over interior nodes: the
  vertex-quadrature L2 norm used by the accuracy gate.
* Energy norm ||v||_a = (v^T A v)^{1/2} (Section 2, after eq. "coercive").
* Element-quadrature L2 and H1-seminorm errors of a P1 function against an
  exact u and grad u, for the rates of Lemma 2.1 and Corollary 3.1
  (O(h^2) in L2, O(h) in energy).  The element rule is a collapsed
  (Duffy) tensor Gauss-Legendre rule, accurate far beyond the P1 error.
"""
from __future__ import annotations

import math

import numpy as np

from .fem import simplex_geometry
from .mesh import Mesh


def nodal_l2(m: np.ndarray, v: np.ndarray) -> float:
    return float(np.sqrt(np.sum(m * v * v)))


def energy_norm(A, v: np.ndarray) -> float:
    return float(np.sqrt(max(float(v @ (A @ v)), 0.0)))


def _collapsed_rule(d: int, npts: int):
    """Points (barycentric, (Q, d+1)) and weights (sum = 1/d!) on the reference simplex."""
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    if d == 2:
        U, V = np.meshgrid(x, x, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        px, py = U * (1 - V), U * V
        wt = WU * WV * U
        pts = np.stack([px.ravel(), py.ravel()], 1)
    elif d == 3:
        U, V, W = np.meshgrid(x, x, x, indexing="ij")
        WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
        px, py, pz = U * (1 - V), U * V * (1 - W), U * V * W
        wt = WU * WV * WW * U * U * V
        pts = np.stack([px.ravel(), py.ravel(), pz.ravel()], 1)
    else:
        raise ValueError(d)
    bary = np.concatenate([1.0 - pts.sum(1, keepdims=True), pts], axis=1)
    return bary, wt.ravel()


def element_errors(mesh: Mesh, u_nodes_full: np.ndarray, u_exact, grad_exact,
                   npts: int = 4, chunk: int = 200_000):
    """(L2 error, H1-seminorm error) of the P1 interpolant of u_nodes_full."""
    d = mesh.dim
    bary, wref = _collapsed_rule(d, npts)
    fact = math.factorial(d)
    e0 = 0.0
    e1 = 0.0
    T = mesh.simplices
    for s in range(0, T.shape[0], chunk):
        Ts = T[s:s + chunk]
        X = mesh.coords[Ts]                                # (E, d+1, d)
        grads, vol, _ = simplex_geometry(X)
        uv = u_nodes_full[Ts]                              # (E, d+1)
        pts = np.einsum("qi,eia->eqa", bary, X)            # (E, Q, d)
        uh = uv @ bary.T                                   # (E, Q)
        ue = u_exact(*[pts[..., a] for a in range(d)])
        gh = np.einsum("ei,eia->ea", uv, grads)            # (E, d)
        ge = grad_exact(*[pts[..., a] for a in range(d)])
        wq = wref[None, :] * (vol * fact)[:, None]          # (E, Q)
        e0 += float(np.sum(wq * (ue - uh) ** 2))
        gsq = sum((ge[a] - gh[:, a:a + 1]) ** 2 for a in range(d))
        e1 += float(np.sum(wq * gsq))
    return math.sqrt(e0), math.sqrt(e1)
