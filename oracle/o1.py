"""Oracle O1: the exact discrete solution of eq. "FEM_form" (Section 2).

Find U (interior nodal values of u_h in V_h) with
    A U + M f(U) = M g,        M = diag(m_j) (vertex quadrature),
by damped Newton on the fine space: J = A + M diag(f'(U)), sparse direct
solves (SuperLU) for the Newton systems, conjugate gradients beyond about a
million unknowns.  This is the unique solution ubar_h of Lemma 2.1; it is
also the fixed point of the correction step of Algorithm 3.1 (if the input
is ubar_h, the linearised problem's solution and every multigrid iterate stay
at ubar_h, and ubar_h solves the augmented problem), so repeated correction
steps converge to it.

Stopping: ||dU||_2 <= tol ||U||_2 or stagnation of ||dU|| (update norms, not
residual norms, because the relative residual has a rounding floor near
1e-10 at a few million unknowns).

With coef (the matrix A(x) per cell, oracle/fem.py) the operator is
-div(A grad u); with f_weight (c at every node, c >= 0) the nonlinearity is
f(x, u) = c(x) f(u), taken by the vertex rule as m_j c_j f(U_j).

With quadrature="element" the pairings use the degree-2 element rule of
oracle/quadrature.py instead: A U + N(U) = G with N_i = (f(u_h), phi_i),
G_i = (g_I, phi_i), and Newton matrix A + K(f'(u_h)) (the f'-weighted mass
matrix of the same rule).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import assemble_interior
from .mesh import Mesh, unit_mesh
from .newton import newton_minimize
from .nonlinear import Nonlinearity
from .quadrature import ElementQuadrature, full_vector

DIRECT_LIMIT = 1_200_000


@dataclass
class O1Result:
    U: np.ndarray            # interior values
    iterations: int
    converged: bool
    mesh: Mesh
    A: sp.csr_matrix
    m: np.ndarray

    def full(self) -> np.ndarray:
        """Nodal values on all (n+1)^d nodes, boundary = 0."""
        out = np.zeros(self.mesh.coords.shape[0])
        out[self.mesh.interior] = self.U
        return out


def _linear_solver(dim, N):
    """SuperLU (symmetric minimum-degree ordering) for 2D up to ~1M unknowns and
    tiny 3D systems; conjugate gradients (J is SPD) otherwise."""
    if (dim == 2 and N <= DIRECT_LIMIT) or N <= 5000:
        def solve(J, R):
            return spla.splu(J.tocsc(), permc_spec="MMD_AT_PLUS_A").solve(R)
    else:
        def solve(J, R):
            x, info = spla.cg(J, R, rtol=1e-14, maxiter=50000)
            if info != 0:
                raise RuntimeError(f"CG did not converge ({info})")
            return x
    return solve


def solve_fine(dim: int, n: int, g_nodes: np.ndarray, nl: Nonlinearity,
               U0=None, tol: float = 1e-14, max_iter: int = 60,
               mesh: Mesh | None = None, A=None, m=None, quadrature: str = "vertex",
               coef=None, f_weight=None) -> O1Result:
    """ubar_h on the (0,1)^dim mesh with n cells per side; g (and c) at all nodes."""
    mesh = mesh if mesh is not None else unit_mesh(dim, n)
    if A is None or m is None:
        A, m = assemble_interior(mesh, coef)
    N = mesh.interior.size
    if quadrature == "vertex":
        g = np.asarray(g_nodes, dtype=np.float64)[mesh.interior]
        mg = m * g
        mc = m if f_weight is None else m * np.asarray(f_weight, dtype=np.float64)[mesh.interior]

        def grad_hess(U):
            R = A @ U + mc * nl.f(U) - mg
            J = (A + sp.diags(mc * nl.df(U))).tocsr()
            return R, J

        def energy(U):
            t1 = 0.5 * float(U @ (A @ U))
            t2 = float(mc @ nl.F(U))
            t3 = float(mg @ U)
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)
    elif quadrature == "element":
        if f_weight is not None:
            raise ValueError("the element rule is read with c = 1 only")
        I = mesh.interior
        Qd = ElementQuadrature(mesh)
        mg = Qd.load(g_nodes)[I]

        def grad_hess(U):
            uf = full_vector(mesh, U)
            R = A @ U + Qd.nonlinear(uf, nl)[I] - mg
            J = (A + Qd.jacobian(uf, nl)[I][:, I]).tocsr()
            return R, J

        def energy(U):
            t1 = 0.5 * float(U @ (A @ U))
            t2 = Qd.energy(full_vector(mesh, U), nl)
            t3 = float(mg @ U)
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)
    else:
        raise ValueError(quadrature)

    def converged(step, U):
        return np.linalg.norm(step) <= tol * max(np.linalg.norm(U), 1e-300)

    U0 = np.zeros(N) if U0 is None else np.asarray(U0, dtype=np.float64)
    U, it, ok = newton_minimize(U0, grad_hess, energy, _linear_solver(dim, N), converged,
                                max_iter=max_iter)
    return O1Result(U, it, ok, mesh, A, m)


def discrete_residual(A, m, U, g_int, nl: Nonlinearity) -> np.ndarray:
    """R(U) = A U + M f(U) - M g (interior), in float64."""
    return A @ U + m * nl.f(U) - m * g_int
