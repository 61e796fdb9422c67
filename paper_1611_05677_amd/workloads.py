"""Seeded synthetic problem data for the semilinear model problem.

This module only *describes problems*: the domain (0,1)^d, mesh depth, the
nonlinearity's catalogue name, and nodal samples of the load g (and of the
manufactured exact solution u where one exists).  It contains none of the
solver's arithmetic; both the CPU oracle and the GPU path take their inputs
from here and from nowhere else.

Problem statement (Section 2, eq. "semilinear equation"):
    -Laplace(u) + f(u) = g in Omega = (0,1)^d,  u = 0 on the boundary.

Manufactured problems follow the paper's examples (Section 4, Examples 1-3)
and the benchmark configurations built from them:
    * u = sin(pi x) sin(pi y)                 2D, f = u^3
    * u = sin(pi x) sin(pi y) exp(x)          2D, f = u^3
    * u = sin(pi x) sin(pi y) sin(pi z)       3D, f = u + sin(u)  (or u^3, Example 1)
    * u = sin(2 pi x) sin(2 pi y) sin(2 pi z) 3D, f = sign(u)|u|^{3/2} (Example 3)
    * g = 1, f = -exp(-u)                     3D, no closed form (Example 2)
g is obtained by applying -Laplace + f to u in closed form.

Random loads: g(x) = sum_{k in {1..K}^d} c_k prod_i sin(k_i pi x_i) with
c_k = xi_k / (1 + |k|^2), xi_k ~ N(0,1) i.i.d. (numpy PCG64, seeded).

Nodal arrays have (n+1)^d entries with x varying fastest (then y, then z);
boundary entries are included (the solvers ignore them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

PI = math.pi

# Catalogue names shared by the oracle and the GPU binding (the integer codes
# are the C ABI's; see include/fmg.h).
F_ZERO, F_LINEAR, F_CUBIC, F_U_PLUS_SIN, F_ABS_U_U, F_SIGNED_POW, F_NEG_EXP = range(7)
F_NAMES = {
    F_ZERO: "zero", F_LINEAR: "linear", F_CUBIC: "cubic", F_U_PLUS_SIN: "u_plus_sin",
    F_ABS_U_U: "abs_u_u", F_SIGNED_POW: "signed_pow", F_NEG_EXP: "neg_exp",
}


def grid_coords(d: int, n: int) -> list[np.ndarray]:
    """1-D node coordinates i/n, i = 0..n, for each axis (same on every axis)."""
    return [np.arange(n + 1, dtype=np.float64) / n for _ in range(d)]


def _outer(vals: list[np.ndarray]) -> np.ndarray:
    """Tensor product of per-axis factors, flattened with x fastest.

    vals[0] is the x factor, vals[1] the y factor (and vals[2] the z factor).
    """
    out = vals[0]
    for v in vals[1:]:
        out = np.multiply.outer(v, out)  # new slower axis in front
    return out.reshape(-1)


def _mesh(d: int, n: int) -> list[np.ndarray]:
    """Full coordinate arrays (x fastest), each of length (n+1)^d."""
    t = np.arange(n + 1, dtype=np.float64) / n
    shape = (n + 1,) * d
    idx = np.indices(shape)  # idx[0] is the slowest axis
    return [t[idx[d - 1 - a]].reshape(-1) for a in range(d)]


def _f_closed(kind: int, param: float, u: np.ndarray) -> np.ndarray:
    """Nonlinearity value used only to manufacture g from an exact u."""
    if kind == F_ZERO:
        return np.zeros_like(u)
    if kind == F_LINEAR:
        return param * u
    if kind == F_CUBIC:
        return u ** 3
    if kind == F_U_PLUS_SIN:
        return u + np.sin(u)
    if kind == F_ABS_U_U:
        return np.abs(u) * u
    if kind == F_SIGNED_POW:
        return np.sign(u) * np.abs(u) ** param
    if kind == F_NEG_EXP:
        return -np.exp(-u)
    raise ValueError(kind)


@dataclass
class Problem:
    """One synthetic instance: mesh depth, nonlinearity and the load g."""
    name: str
    dim: int
    coarse_cells: int
    refinements: int
    f_kind: int
    f_param: float
    g_nodes: np.ndarray                  # (n+1)^d, x fastest
    u_exact_nodes: Optional[np.ndarray] = None
    u_exact: Optional[Callable] = None   # u(*coords) -> array, for element norms
    grad_u_exact: Optional[Callable] = None
    meta: dict = field(default_factory=dict)
    # variable coefficients: the symmetric positive definite matrix A per cell
    # of the finest mesh as its d(d+1)/2 upper-triangle components row by row
    # (2D: a11, a12, a22; 3D: a11, a12, a13, a22, a23, a33), shape
    # (components, n^d), cells x fastest by lower corner; and the weight
    # c >= 0 of f(x, u) = c(x) f(u) at the finest nodes ((n+1)^d).  None: A = I, c = 1
    coef_cells: Optional[np.ndarray] = None
    f_weight_nodes: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.coarse_cells * 2 ** self.refinements

    @property
    def n_levels(self) -> int:
        return self.refinements + 1

    @property
    def interior_dofs(self) -> int:
        return (self.n - 1) ** self.dim


# ---------------------------------------------------------------------------
# Manufactured solutions: u, grad u and -Laplace(u) in closed form.
# ---------------------------------------------------------------------------

def _sines(d: int, freq: float):
    def u(*x):
        out = np.ones_like(x[0])
        for xi in x:
            out = out * np.sin(freq * PI * xi)
        return out

    def grad(*x):
        g = []
        for a in range(d):
            term = freq * PI * np.cos(freq * PI * x[a])
            for b in range(d):
                if b != a:
                    term = term * np.sin(freq * PI * x[b])
            g.append(term)
        return g

    def neg_lap(*x):
        return d * (freq * PI) ** 2 * u(*x)

    return u, grad, neg_lap


def _sines_expx():
    """u = sin(pi x) sin(pi y) exp(x) on the unit square."""
    def u(x, y):
        return np.sin(PI * x) * np.sin(PI * y) * np.exp(x)

    def grad(x, y):
        ex = np.exp(x)
        return [ex * np.sin(PI * y) * (np.sin(PI * x) + PI * np.cos(PI * x)),
                PI * ex * np.sin(PI * x) * np.cos(PI * y)]

    def neg_lap(x, y):
        ex = np.exp(x)
        return ex * np.sin(PI * y) * ((2 * PI ** 2 - 1) * np.sin(PI * x)
                                      - 2 * PI * np.cos(PI * x))

    return u, grad, neg_lap


MANUFACTURED = {
    "sin": lambda d: _sines(d, 1.0),
    "sin2": lambda d: _sines(d, 2.0),
    "sin_expx": lambda d: _sines_expx(),
}


def manufactured(name: str, dim: int, coarse_cells: int, refinements: int,
                 solution: str, f_kind: int, f_param: float = 0.0) -> Problem:
    """g = -Laplace(u) + f(u) for a closed-form u, sampled at the finest nodes."""
    u, grad, neg_lap = MANUFACTURED[solution](dim)
    n = coarse_cells * 2 ** refinements
    X = _mesh(dim, n)
    un = u(*X)
    g = neg_lap(*X) + _f_closed(f_kind, f_param, un)
    return Problem(name, dim, coarse_cells, refinements, f_kind, f_param,
                   g_nodes=np.ascontiguousarray(g), u_exact_nodes=un,
                   u_exact=u, grad_u_exact=grad,
                   meta={"solution": solution})


def constant_load(name: str, dim: int, coarse_cells: int, refinements: int,
                  value: float, f_kind: int, f_param: float = 0.0) -> Problem:
    n = coarse_cells * 2 ** refinements
    g = np.full((n + 1) ** dim, float(value))
    return Problem(name, dim, coarse_cells, refinements, f_kind, f_param, g_nodes=g,
                   meta={"load": value})


def fourier_coefficients(dim: int, modes: int, seed) -> np.ndarray:
    """c_k = xi_k / (1 + |k|^2), k in {1..modes}^dim, xi ~ N(0,1) from PCG64(seed).

    Returned with axis a holding k_{a+1} (so c[k1-1, k2-1] in 2D).
    """
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((modes,) * dim)
    k = np.arange(1, modes + 1, dtype=np.float64)
    ksq = np.zeros((modes,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = modes
        ksq = ksq + (k ** 2).reshape(shape)
    return xi / (1.0 + ksq)


def fourier_load_nodes(coef: np.ndarray, n: int) -> np.ndarray:
    """Evaluate sum_k c_k prod_a sin(k_a pi x_a) at the (n+1)^d nodes (x fastest)."""
    dim = coef.ndim
    modes = coef.shape[0]
    t = np.arange(n + 1, dtype=np.float64) / n
    k = np.arange(1, modes + 1, dtype=np.float64)
    S = np.sin(PI * np.outer(k, t))  # (modes, n+1): S[k-1, i] = sin(k pi t_i)
    if dim == 2:
        # G[j, i] = sum_{k1,k2} c[k1,k2] S[k1,i] S[k2,j]  (x = axis of k1)
        G = S.T @ coef.T @ S  # (n+1 [y], n+1 [x])
        return np.ascontiguousarray(G.reshape(-1))
    if dim == 3:
        # G[l, j, i] = sum c[k1,k2,k3] S[k1,i] S[k2,j] S[k3,l]
        T1 = np.einsum("abc,ai->ibc", coef, S)      # contract k1 -> x
        T2 = np.einsum("ibc,bj->ijc", T1, S)        # contract k2 -> y
        G = np.einsum("ijc,cl->lji", T2, S)         # contract k3 -> z; order (z,y,x)
        return np.ascontiguousarray(G.reshape(-1))
    raise ValueError(dim)


def fourier_load_device(coef: np.ndarray, n: int, device, stream=None):
    """fourier_load_nodes evaluated with torch float64 products on `device`
    (same sums, possibly another rounding order).  Used where loads are made
    per request on the GPU instead of being shipped from the host."""
    import torch
    dim = coef.ndim
    modes = coef.shape[0]
    t = torch.arange(n + 1, dtype=torch.float64, device=device) / n
    k = torch.arange(1, modes + 1, dtype=torch.float64, device=device)
    S = torch.sin(PI * torch.outer(k, t))                      # (modes, n+1)
    C = torch.as_tensor(coef, dtype=torch.float64).to(device)
    if dim == 2:
        G = S.t().contiguous() @ C.t().contiguous() @ S       # (y, x)
        return G.reshape(-1).contiguous()
    if dim == 3:
        m, N = modes, n + 1
        St = S.t().contiguous()                                # (N, m)
        X = (St @ C.reshape(m, m * m)).reshape(N, m, m)        # X[i, b, c]
        Y = (X.permute(0, 2, 1).contiguous().reshape(N * m, m) @ S).reshape(N, m, N)   # Y[i, c, j]
        Z = (Y.permute(0, 2, 1).contiguous().reshape(N * N, m) @ S).reshape(N, N, N)   # Z[i, j, l]
        return Z.permute(2, 1, 0).contiguous().reshape(-1)     # (l, j, i): x fastest
    raise ValueError(dim)


def fourier_problem(name: str, dim: int, coarse_cells: int, refinements: int,
                    f_kind: int, seed, modes: int = 16, f_param: float = 0.0) -> Problem:
    coef = fourier_coefficients(dim, modes, seed)
    n = coarse_cells * 2 ** refinements
    return Problem(name, dim, coarse_cells, refinements, f_kind, f_param,
                   g_nodes=fourier_load_nodes(coef, n),
                   meta={"modes": modes, "seed": seed})


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------

def square_cubic_sin(refinements: int = 5) -> Problem:
    """2D unit square, f = u^3, u = sin(pi x) sin(pi y); 4x4 coarse grid."""
    return manufactured(f"square_cubic_sin_L{refinements}", 2, 4, refinements, "sin", F_CUBIC)


def square_cubic_sin_expx(refinements: int = 9) -> Problem:
    """2D unit square, f = u^3, u = sin(pi x) sin(pi y) exp(x); 4x4 coarse grid."""
    return manufactured(f"square_cubic_sin_expx_L{refinements}", 2, 4, refinements,
                        "sin_expx", F_CUBIC)


def cube_u_plus_sin(refinements: int = 6) -> Problem:
    """3D unit cube (Kuhn tetrahedra), f = u + sin u, u = sin sin sin; 4^3 coarse grid."""
    return manufactured(f"cube_u_plus_sin_L{refinements}", 3, 4, refinements, "sin", F_U_PLUS_SIN)


def cube_example1(refinements: int) -> Problem:
    """Section 4, Example 1: f = u^3, u = sin(pi x) sin(pi y) sin(pi z)."""
    return manufactured(f"cube_example1_L{refinements}", 3, 4, refinements, "sin", F_CUBIC)


def cube_example3(refinements: int) -> Problem:
    """Section 4, Example 3: f = sign(u)|u|^{3/2}, u = sin(2 pi x) sin(2 pi y) sin(2 pi z)."""
    return manufactured(f"cube_example3_L{refinements}", 3, 4, refinements, "sin2",
                        F_SIGNED_POW, 1.5)


def cube_example2(refinements: int) -> Problem:
    """Section 4, Example 2: -Laplace(u) - exp(-u) = 1, no closed-form solution."""
    return constant_load(f"cube_example2_L{refinements}", 3, 4, refinements, 1.0, F_NEG_EXP)


# Batched workload: 64 independent 2D problems, depths U{6..10}, f = u^3,
# random 16x16-mode loads.
BATCH_SEED = 161105677


def batched_specs(count: int = 64, depth_lo: int = 6, depth_hi: int = 10,
                  seed: int = BATCH_SEED) -> list[tuple[int, list]]:
    """(depth, coefficient seed) of each problem of the batched workload."""
    rng = np.random.default_rng(seed)
    depths = rng.integers(depth_lo, depth_hi + 1, size=count)
    return [(int(depths[i]), [seed, i]) for i in range(count)]


def batched_problems(count: int = 64, depth_lo: int = 6, depth_hi: int = 10,
                     seed: int = BATCH_SEED) -> list[Problem]:
    return [fourier_problem(f"batch_{i}", 2, 4, d, F_CUBIC, sd)
            for i, (d, sd) in enumerate(batched_specs(count, depth_lo, depth_hi, seed))]


# Served workload: Poisson arrivals (rate 200/s) of mixed 2D/3D solves.
SERVE_SEED = 161105678
SERVE_KINDS = (F_CUBIC, F_U_PLUS_SIN, F_ABS_U_U)


@dataclass
class Request:
    rid: int
    arrival_s: float
    dim: int
    refinements: int
    f_kind: int
    seed: list


def serving_trace(count: int = 4000, rate_hz: float = 200.0, seed: int = SERVE_SEED,
                  depths2d=(7, 10), depths3d=(3, 6)) -> list[Request]:
    """Open-loop arrival trace: exponential gaps, per-request dim/depth/f uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    dims = rng.integers(2, 4, size=count)
    out = []
    for i in range(count):
        lo, hi = depths2d if dims[i] == 2 else depths3d
        depth = int(rng.integers(lo, hi + 1))
        kind = int(SERVE_KINDS[rng.integers(0, len(SERVE_KINDS))])
        out.append(Request(i, float(t[i]), int(dims[i]), depth, kind, [seed, i]))
    return out


def request_problem(req: Request, modes: int = 16) -> Problem:
    return fourier_problem(f"req_{req.rid}", req.dim, 4, req.refinements, req.f_kind,
                           req.seed, modes=modes)


# Random linear functionals for comparing long nodal vectors: row i of the
# sketch is a vector of i.i.d. N(0,1) weights from PCG64([seed, i]).  For any
# difference vector e, the mean of (w_i . e)^2 over the rows estimates |e|^2,
# so agreement of a few such functionals checks a whole vector, not a sample.
SKETCH_SEED = 20161118
SKETCH_ROWS = 16


def sketch_row(count: int, i: int, seed: int = SKETCH_SEED) -> np.ndarray:
    """Weights of sketch row i for vectors of `count` entries."""
    return np.random.default_rng([seed, i]).standard_normal(count)


# ---------------------------------------------------------------------------
# Variable coefficients: -div(kappa grad u) + c(x) f(u) = g.
# ---------------------------------------------------------------------------

def _cell_centres(d: int, n: int) -> list[np.ndarray]:
    """Centre coordinates of the n^d cells (x fastest), one array per axis."""
    t = (np.arange(n, dtype=np.float64) + 0.5) / n
    idx = np.indices((n,) * d)
    return [t[idx[d - 1 - a]].reshape(-1) for a in range(d)]


def _upper_components(M: np.ndarray) -> list[tuple[int, int]]:
    d = M.shape[0]
    return [(a, b) for a in range(d) for b in range(a, d)]


# Constant anisotropy of the manufactured variable-coefficient problems
# (symmetric, diagonally dominant, so positive definite).
ANISO = {2: np.array([[1.0, 0.3], [0.3, 0.8]]),
         3: np.array([[1.0, 0.3, 0.2], [0.3, 0.9, 0.25], [0.2, 0.25, 1.1]])}


def scalar_coefficient(dim: int, kappa: np.ndarray) -> np.ndarray:
    """Components (d(d+1)/2, cells) of A = kappa I."""
    kappa = np.asarray(kappa, dtype=np.float64)
    return np.stack([kappa if a == b else np.zeros_like(kappa)
                     for a, b in _upper_components(np.eye(dim))])


def variable_coefficient(name: str, dim: int, coarse_cells: int, refinements: int,
                         f_kind: int, f_param: float = 0.0, isotropic: bool = False) -> Problem:
    """u = s = prod sin(pi x_i), A(x) = kappa(x) B with kappa = 1 + s/2 sampled
    at the cell centres and B = ANISO[dim] (or I), c(x) = 1 + cos(pi x_1)/2 at
    the nodes, and g = -div(A grad u) + c f(u) in closed form at the nodes:
    -kappa tr(B H_s) - (grad kappa)^T B grad s + c f(s), H_s the Hessian of s."""
    B = np.eye(dim) if isotropic else ANISO[dim]
    n = coarse_cells * 2 ** refinements
    X = _mesh(dim, n)
    S = [np.sin(PI * x) for x in X]
    Cs = [np.cos(PI * x) for x in X]
    s_ = np.prod(S, axis=0)

    def prod_except(*skip):
        out = np.ones_like(X[0])
        for k in range(dim):
            if k not in skip:
                out = out * S[k]
        return out

    grad = [PI * Cs[a] * prod_except(a) for a in range(dim)]
    trBH = np.zeros_like(X[0])
    for a in range(dim):
        for b in range(dim):
            Hab = -PI ** 2 * s_ if a == b else PI ** 2 * Cs[a] * Cs[b] * prod_except(a, b)
            trBH += B[a, b] * Hab
    gBg = sum(B[a, b] * grad[a] * grad[b] for a in range(dim) for b in range(dim))
    kap_nodes = 1.0 + 0.5 * s_
    c = 1.0 + 0.5 * np.cos(PI * X[0])
    g = -kap_nodes * trBH - 0.5 * gBg + c * _f_closed(f_kind, f_param, s_)
    C = _cell_centres(dim, n)
    kc = 1.0 + 0.5 * np.prod([np.sin(PI * x) for x in C], axis=0)
    coef = np.stack([kc * B[a, b] for a, b in _upper_components(B)])
    return Problem(name, dim, coarse_cells, refinements, f_kind, f_param, g_nodes=np.ascontiguousarray(g),
                   u_exact_nodes=s_, coef_cells=np.ascontiguousarray(coef),
                   f_weight_nodes=np.ascontiguousarray(c),
                   meta={"solution": "sin", "A": "(1 + s/2) " + ("I" if isotropic else "B")})


def random_coefficient(name: str, dim: int, coarse_cells: int, refinements: int, f_kind: int, seed,
                       contrast: float = 10.0, f_param: float = 0.0) -> Problem:
    """A = kappa (I + 0.4 S) per cell: kappa log-uniform in [1, contrast], S
    symmetric with zero diagonal and off-diagonal entries uniform in
    [-1/2, 1/2] (eigenvalues of I + 0.4 S >= 0.6); c uniform in [0, 2] at the
    nodes; a random-Fourier load (PCG64 seeded)."""
    rng = np.random.default_rng(seed)
    n = coarse_cells * 2 ** refinements
    P = fourier_problem(name, dim, coarse_cells, refinements, f_kind, [int(x) for x in np.atleast_1d(seed)] + [7],
                        f_param=f_param)
    ncell = n ** dim
    kappa = np.exp(rng.uniform(0.0, np.log(contrast), size=ncell))
    comps = []
    for a, b in _upper_components(np.eye(dim)):
        comps.append(kappa if a == b else kappa * 0.4 * rng.uniform(-0.5, 0.5, size=ncell))
    P.coef_cells = np.ascontiguousarray(np.stack(comps))
    P.f_weight_nodes = rng.uniform(0.0, 2.0, size=(n + 1) ** dim)
    P.meta.update({"A": f"kappa (I + 0.4 S), kappa log-uniform [1, {contrast:g}] per cell",
                   "c": "uniform [0, 2] per node"})
    return P
