"""Oracle O2: the full multigrid scheme, replicated plainly on the CPU.

Section 3, Algorithm 3.1 (one correction step, "SemilinearMG") and
Algorithm 3.2 (full multigrid scheme), with CSR stiffness matrices assembled
element by element on every level and sparse prolongations P_k built by point
location (barycentric coordinates of the fine nodes in the coarse simplices).

Readings of what the paper leaves open (shared with the GPU library):
  * V_H = V_{h_1}: the coarsest mesh (n_H cells per side) is the coarse space of
    the augmented problem, so Algorithm 3.2 runs on levels k = 1..n with
    n = refinements + 1.
  * "m multigrid iteration steps" (eq. "Error_Reduction") are V(nu1, nu2)
    cycles started from u^(l): damped-Jacobi sweeps x <- x + w_i D^{-1}(b - A x)
    with D = diag(A_k); residual restriction by P_k^T; exact solve on level 1;
    correction by P_k; post-sweeps with the weights in reverse order.  Default
    weights: 2D w = 4/5 every sweep; 3D the degree-nu Chebyshev weights for
    D^{-1}A on [1/3, 2], w_i = 1/(c + r cos(pi (2i-1)/(2 nu))), c = 7/6, r = 5/6.
  * All L2 pairings use vertex quadrature on the current finest level k,
    including those of the augmented problem eq. "coarse problem"; with
    Options.quadrature = "element" they use instead the degree-2 element rule
    of oracle/quadrature.py on the level-k simplices, everywhere: the
    linearised load (g - f(u^(l)), v), the augmented problem, and level 1.
  * The augmented problem is solved by damped Newton in the coordinates
    (w, alpha) of z = Q_k w + alpha u~ (Q_k = P_k ... P_2), started at
    (0, 1), i.e. z = u~ (the good initial guess of the Remark after
    Theorem 3.3), and stopped as soon as a Newton direction (applied in full)
    or an accepted damped update d satisfies |d|_inf <= tol max(1, |w|_inf, |alpha|).
  * If u~ adds (numerically) nothing to V_H -- the Schur complement of the
    alpha row of the Newton matrix is <= 1e-12 of its diagonal entry -- the
    alpha component of the step is set to zero and the w block solved alone.
  * Level 1 (Algorithm 3.2, step 1) is solved by the same Newton iteration.
  * Variable coefficient (A(x) symmetric positive definite, constant on every
    cell of the finest mesh): a(u, v) is one form on all the nested spaces, so
    the matrix of level k is that form on V_{h_k}, A_k = P_{k+1}^T A_{k+1}
    P_{k+1} down from the finest assembly (with A = I this is the plain
    assembly on every level).  An x-dependent f(x, u) = c(x) f(u) takes c at
    the level's nodes (nodes of the finest mesh), in the vertex rule
    m_j c_j f(u_j).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .fem import assemble_interior, prolongation
from .mesh import Mesh, unit_mesh
from .newton import newton_minimize
from .nonlinear import Nonlinearity
from .quadrature import ElementQuadrature, full_vector

JACOBI, CHEBYSHEV = 1, 2
SCHUR_DROP = 1e-12
# Converged mode: an update that no longer shrinks ends the iteration; it counts
# as converged only if the relative update is within this factor of the
# tolerance (rounding level), and as not converged otherwise.
STAGNATION_FLOOR = 1e3


def chebyshev_weights(nu: int, lo: float, hi: float) -> list[float]:
    """Reciprocals of the roots of the degree-nu Chebyshev polynomial on [lo, hi]."""
    c, r = 0.5 * (hi + lo), 0.5 * (hi - lo)
    return [1.0 / (c + r * math.cos(math.pi * (2 * i - 1) / (2 * nu))) for i in range(1, nu + 1)]


@dataclass
class Options:
    m_vcycles: int = 2          # "m" of Algorithm 3.1 (Section 4 uses m = 2)
    p_steps: int = 1            # "p" of Algorithm 3.2 (Section 4 uses p = 1)
    nu_pre: int = 2
    nu_post: int = 2
    smoother: int = 0           # 0: default for the dimension
    omega: float = 0.0          # Jacobi weight, 0 -> 4/5 (2D) or 6/7 (3D)
    cheb_lo: float = 1.0 / 3.0
    cheb_hi: float = 2.0
    newton_tol: float = 1e-14
    newton_max: int = 30
    converged_tol: float = 1e-13
    converged_max_steps: int = 40
    quadrature: str = "vertex"  # or "element"

    def weights(self, dim: int):
        kind = self.smoother or (JACOBI if dim == 2 else CHEBYSHEV)
        if kind == JACOBI:
            w = self.omega or (4.0 / 5.0 if dim == 2 else 6.0 / 7.0)
            pre = [w] * self.nu_pre
            post = [w] * self.nu_post
        else:
            pre = chebyshev_weights(self.nu_pre, self.cheb_lo, self.cheb_hi)
            post = chebyshev_weights(self.nu_post, self.cheb_lo, self.cheb_hi)[::-1]
        return pre, post


@dataclass
class Level:
    mesh: Mesh
    A: sp.csr_matrix
    m: np.ndarray
    D: np.ndarray
    P: sp.csr_matrix | None = None    # from level k-1 to this level
    Q: sp.csr_matrix | None = None    # V_H -> this level


class Hierarchy:
    """Meshes T_{h_1} .. T_{h_n}, matrices A_k, masses m_k, P_k and Q_k."""

    def __init__(self, dim: int, coarse_cells: int, refinements: int, coef=None):
        self.dim = dim
        self.coarse_cells = coarse_cells
        self.levels: list[Level] = []
        for k in range(refinements + 1):
            mesh = unit_mesh(dim, coarse_cells * 2 ** k)
            A, m = assemble_interior(mesh, coef if (coef is None or k == refinements) else None)
            lev = Level(mesh, A, m, A.diagonal().copy())
            if k == 0:
                lev.Q = sp.identity(mesh.interior.size, format="csr")
            else:
                lev.P = prolongation(self.levels[-1].mesh, mesh)
                lev.Q = (lev.P @ self.levels[-1].Q).tocsr()
            self.levels.append(lev)
        if coef is not None:
            # the finest form on the coarser spaces (Galerkin)
            for k in range(refinements - 1, -1, -1):
                P = self.levels[k + 1].P
                A = (P.T @ self.levels[k + 1].A @ P).tocsr()
                A.sort_indices()
                self.levels[k].A = A
                self.levels[k].D = A.diagonal().copy()
        self.A1 = self.levels[0].A.toarray()
        self._quad = {}

    def quad(self, k: int) -> ElementQuadrature:
        """Element rule on the level-k simplices (built on first use)."""
        if k not in self._quad:
            self._quad[k] = ElementQuadrature(self.levels[k].mesh)
        return self._quad[k]

    @property
    def n_levels(self) -> int:
        return len(self.levels)

    def g_on_level(self, g_fine_nodes: np.ndarray, k: int) -> np.ndarray:
        """Nodal g at level-k interior nodes (level-k nodes are fine nodes)."""
        fine = self.levels[-1].mesh
        mesh = self.levels[k].mesh
        s = fine.n // mesh.n
        ids = np.zeros(mesh.interior.size, dtype=np.int64)
        ijk = mesh.ijk[mesh.interior] * s
        for a in range(self.dim - 1, -1, -1):
            ids = ids * (fine.n + 1) + ijk[:, a]
        return np.asarray(g_fine_nodes, dtype=np.float64)[ids]

    def g_full_on_level(self, g_fine_nodes: np.ndarray, k: int) -> np.ndarray:
        """Nodal g at all level-k nodes, boundary nodes included (element rule)."""
        fine = self.levels[-1].mesh
        mesh = self.levels[k].mesh
        s = fine.n // mesh.n
        ids = np.zeros(mesh.coords.shape[0], dtype=np.int64)
        ijk = mesh.ijk * s
        for a in range(self.dim - 1, -1, -1):
            ids = ids * (fine.n + 1) + ijk[:, a]
        return np.asarray(g_fine_nodes, dtype=np.float64)[ids]


# ---------------------------------------------------------------------------
# Linear multigrid (the "m multigrid iteration steps" of Algorithm 3.1, step 1)
# ---------------------------------------------------------------------------

def smooth(lev: Level, x, b, weights):
    for w in weights:
        x = x + w * (b - lev.A @ x) / lev.D
    return x


def vcycle(H: Hierarchy, k: int, x, b, pre, post):
    if k == 0:
        return np.linalg.solve(H.A1, b)
    lev = H.levels[k]
    x = smooth(lev, x, b, pre)
    r = b - lev.A @ x
    bc = lev.P.T @ r
    xc = vcycle(H, k - 1, np.zeros_like(bc), bc, pre, post)
    x = x + lev.P @ xc
    return smooth(lev, x, b, post)


# ---------------------------------------------------------------------------
# Small Newton solves
# ---------------------------------------------------------------------------

def _small_converged(tol):
    def conv(step, y):
        return np.max(np.abs(step)) <= tol * max(1.0, float(np.max(np.abs(y))))
    return conv


def _solve_dense(J, R):
    return np.linalg.solve(J, R)


def _solve_augmented(J, R):
    """Newton system of the augmented problem, dropping the u~ direction when it
    adds nothing to V_H (Schur complement of the last row tiny)."""
    JHH, JHu, Juu = J[:-1, :-1], J[:-1, -1], J[-1, -1]
    y = np.linalg.solve(JHH, JHu)
    schur = Juu - JHu @ y
    if not (schur > SCHUR_DROP * Juu):
        out = np.zeros_like(R)
        out[:-1] = np.linalg.solve(JHH, R[:-1])
        return out
    return np.linalg.solve(J, R)


def level1_solve(H: Hierarchy, g1: np.ndarray, nl: Nonlinearity, opts: Options,
                 g1_full: np.ndarray | None = None, c1: np.ndarray | None = None):
    """Algorithm 3.2, step 1: a(u, v) + (f(u), v) = (g, v) on V_{h_1}.
    g1: interior nodal load; g1_full: load at all level-1 nodes (element rule)."""
    lev = H.levels[0]
    A, m = H.A1, lev.m
    if opts.quadrature == "element":
        Qd, mesh = H.quad(0), lev.mesh
        I = mesh.interior
        mg = Qd.load(g1_full)[I]

        def grad_hess(U):
            uf = full_vector(mesh, U)
            return A @ U + Qd.nonlinear(uf, nl)[I] - mg, A + Qd.jacobian(uf, nl)[I][:, I].toarray()

        def energy(U):
            t1, t2, t3 = 0.5 * U @ A @ U, Qd.energy(full_vector(mesh, U), nl), mg @ U
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)
    else:
        mg = m * g1
        mc = m if c1 is None else m * c1

        def grad_hess(U):
            return A @ U + mc * nl.f(U) - mg, A + np.diag(mc * nl.df(U))

        def energy(U):
            t1, t2, t3 = 0.5 * U @ A @ U, mc @ nl.F(U), mg @ U
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)

    U, it, ok = newton_minimize(np.zeros(A.shape[0]), grad_hess, energy, _solve_dense,
                                _small_converged(opts.newton_tol), opts.newton_max,
                                stagnation=False)
    return U, it, ok


def augmented_solve(H: Hierarchy, k: int, ut: np.ndarray, g_k: np.ndarray,
                    nl: Nonlinearity, opts: Options, g_full: np.ndarray | None = None,
                    c_k: np.ndarray | None = None):
    """Algorithm 3.1, step 2: solve eq. "coarse problem" on V_H + span{u~}.

    Basis B = [Q_k, u~] (columns are fine nodal vectors), z = B y, y = (w, alpha).
    R(y) = B^T (A z + M f(z) - M g), J(y) = B^T (A + M diag f'(z)) B
    (element rule: B^T (A z + N(z) - G) and B^T (A + K(f'(z))) B).
    """
    lev = H.levels[k]
    A, m, Q = lev.A, lev.m, lev.Q
    B = sp.hstack([Q, sp.csr_matrix(ut.reshape(-1, 1))]).tocsr()
    BtAB = (B.T @ (A @ B)).toarray()
    if opts.quadrature == "element":
        Qd, mesh = H.quad(k), lev.mesh
        I = mesh.interior
        Btmg = B.T @ Qd.load(g_full)[I]

        def grad_hess(y):
            zf = full_vector(mesh, B @ y)
            R = BtAB @ y + B.T @ Qd.nonlinear(zf, nl)[I] - Btmg
            J = BtAB + (B.T @ Qd.jacobian(zf, nl)[I][:, I] @ B).toarray()
            return R, J

        def energy(y):
            t1, t2, t3 = 0.5 * y @ BtAB @ y, Qd.energy(full_vector(mesh, B @ y), nl), Btmg @ y
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)
    else:
        mg = m * g_k
        mc = m if c_k is None else m * c_k
        Btmg = B.T @ mg

        def grad_hess(y):
            z = B @ y
            R = BtAB @ y + B.T @ (mc * nl.f(z)) - Btmg
            J = BtAB + (B.T @ sp.diags(mc * nl.df(z)) @ B).toarray()
            return R, J

        def energy(y):
            z = B @ y
            t1, t2, t3 = 0.5 * y @ BtAB @ y, mc @ nl.F(z), Btmg @ y
            return t1 + t2 - t3, abs(t1) + abs(t2) + abs(t3)

    y0 = np.zeros(Q.shape[1] + 1)
    y0[-1] = 1.0
    y, it, ok = newton_minimize(y0, grad_hess, energy, _solve_augmented,
                                _small_converged(opts.newton_tol), opts.newton_max,
                                stagnation=False)
    return B @ y, y, it, ok


@dataclass
class StepInfo:
    level: int
    newton_iters: int
    newton_ok: bool
    alpha: float


def correction_step(H: Hierarchy, k: int, u: np.ndarray, g_k: np.ndarray,
                    nl: Nonlinearity, opts: Options, info: list | None = None,
                    g_full: np.ndarray | None = None, c_k: np.ndarray | None = None):
    """Algorithm 3.1: u^(l+1) = SemilinearMG(V_H, u^(l), V_{h_k}).
    g_k: interior nodal load; g_full: load at all level-k nodes (element rule)."""
    lev = H.levels[k]
    pre, post = opts.weights(H.dim)
    # Step 1: linearised problem eq. "linearized": a(u^, v) = (g - f(u^(l)), v)
    if opts.quadrature == "element":
        Qd, I = H.quad(k), lev.mesh.interior
        b = Qd.load(g_full)[I] - Qd.nonlinear(full_vector(lev.mesh, u), nl)[I]
    else:
        b = lev.m * (g_k - (nl.f(u) if c_k is None else c_k * nl.f(u)))
    ut = u.copy()
    for _ in range(opts.m_vcycles):
        ut = vcycle(H, k, ut, b, pre, post)
    # Step 2: semilinear problem on V_H + span{u~}
    unew, y, it, ok = augmented_solve(H, k, ut, g_k, nl, opts, g_full, c_k)
    if info is not None:
        info.append(StepInfo(k + 1, it, ok, float(y[-1])))
    return unew, ut


@dataclass
class FMGResult:
    U: np.ndarray                     # interior values on the finest level
    steps: list = field(default_factory=list)
    level1_iters: int = 0
    extra_steps: int = 0
    last_update_rel: float = float("nan")
    converged_ok: bool = True             # converged mode: reached the tolerance
    hierarchy: Hierarchy | None = None

    def full(self) -> np.ndarray:
        mesh = self.hierarchy.levels[-1].mesh
        out = np.zeros(mesh.coords.shape[0])
        out[mesh.interior] = self.U
        return out


def fmg(H: Hierarchy, g_fine_nodes: np.ndarray, nl: Nonlinearity,
        opts: Options | None = None, converged: bool = False,
        f_weight: np.ndarray | None = None) -> FMGResult:
    """Algorithm 3.2 on levels 1..n; optionally keep correcting on level n until
    ||du||_2 <= converged_tol ||u||_2 (converged mode, which tends to ubar_h)."""
    opts = opts or Options()
    res = FMGResult(None, hierarchy=H)
    element = opts.quadrature == "element"

    def g_full(k):
        return H.g_full_on_level(g_fine_nodes, k) if element else None

    if element and f_weight is not None:
        raise ValueError("the element rule is read with c = 1 only")

    def c_on(k):
        return None if f_weight is None else H.g_on_level(f_weight, k)

    u, it, _ = level1_solve(H, H.g_on_level(g_fine_nodes, 0), nl, opts, g_full(0), c_on(0))
    res.level1_iters = it
    for k in range(1, H.n_levels):
        u = H.levels[k].P @ u                     # u^(0) = u_{h_{k-1}}
        g_k, gf = H.g_on_level(g_fine_nodes, k), g_full(k)
        for _ in range(opts.p_steps):
            u, _ = correction_step(H, k, u, g_k, nl, opts, res.steps, gf, c_on(k))
    if converged:
        k = H.n_levels - 1
        g_k, gf = H.g_on_level(g_fine_nodes, k), g_full(k)
        prev = np.inf
        res.converged_ok = False
        for s in range(opts.converged_max_steps):
            unew, _ = correction_step(H, k, u, g_k, nl, opts, None, gf, c_on(k))
            du = np.linalg.norm(unew - u)
            u = unew
            res.extra_steps = s + 1
            res.last_update_rel = du / max(np.linalg.norm(u), 1e-300)
            if res.last_update_rel <= opts.converged_tol:
                res.converged_ok = True
                break
            if du >= prev:
                # the update stopped shrinking: rounding level if it is already
                # small, otherwise the iteration stagnates or diverges
                res.converged_ok = res.last_update_rel <= STAGNATION_FLOOR * opts.converged_tol
                break
            prev = du
    res.U = u
    return res
