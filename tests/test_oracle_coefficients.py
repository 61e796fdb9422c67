"""Pins of the oracle's variable-coefficient reading: -div(A grad u) +
c(x) f(u) = g with A symmetric positive definite and constant on every cell
of the finest mesh, c >= 0 at its nodes; the coarser levels carry the same
form (Galerkin: A_k = P^T A_{k+1} P).  oracle/fem.py and the coef /
f_weight paths of O1 and O2.

What fixes them, independently of the code under test:
  * the Kuhn simplices are orthoschemes: with the chain of a simplex
    0, e_a0, e_a0 + e_a1, .. the barycentric gradients are -e_a0,
    e_a0 - e_a1, .., e_a(d-1) (over h).  For A = kappa I the gradients of
    non-consecutive chain vertices are orthogonal, so only axis edges couple,
    each by -kappa h^(d-2) / d! per simplex in which it is a chain step;
    counting simplices: 2D (kappa of the two cells beside the edge) / 2, 3D
    (2 kappa(p) + kappa(p - e_b) + kappa(p - e_c) + 2 kappa(p - e_b - e_c))
    h / 6 (cells by lower corner; b, c the other two axes);
  * for a 2D matrix (a11, a12, a22) per cell the same gradients give the
    x edge (a11 - a12)/2 per adjacent triangle, the y edge (a22 - a12)/2, and
    the cell's diagonal a12/2 from each of its two triangles;
  * for a constant matrix, the P1 stiffness applied to a quadratic u is the
    lumped mass times -tr(A Hess u) at every interior node (consistency on a
    translation-invariant mesh);
  * on a coarse simplex the coarse hat gradients are constant, so the
    Galerkin matrix of a level is the plain assembly on that level with, on
    each simplex, the volume mean of the finest matrices inside it (point
    location by centroid, explicit loops);
  * A = I gives the constant-coefficient hierarchy; c = 1 is the plain
    problem; c = 0 and linear f reduce O1 to one sparse linear solve;
  * the manufactured smooth problem converges at O(h^2); O2 keeps ubar_h
    fixed and meets the Theorem 3.2 gate with the coefficients.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fem import assemble_full, assemble_interior, coefficient_tensors, local_rows
from oracle.mesh import unit_mesh
from oracle.nonlinear import Nonlinearity
from oracle.norms import nodal_l2
from oracle.o1 import solve_fine
from oracle.o2 import Hierarchy, Options, augmented_solve, correction_step, fmg
from paper_1611_05677_amd import workloads as W


def _interior_ids(d, n):
    """Interior node (x, y[, z]) -> dense index, x fastest."""
    pts = [p[::-1] for p in itertools.product(range(1, n), repeat=d)]   # slowest axis first
    return {p: i for i, p in enumerate(pts)}


def _stencil_from_edges(d, n, edges):
    """Interior matrix from forward edge weights: edges(p, delta) -> weight of
    the edge from node p to p + delta (delta a 0/1 tuple, p may be a boundary
    node); A_ii = sum of the weights of all edges at i, A_ij = -weight."""
    ids = _interior_ids(d, n)
    deltas = [dl for dl in itertools.product((0, 1), repeat=d) if any(dl)]
    A = sp.lil_matrix((len(ids), len(ids)))
    for p, i in ids.items():
        for dl in deltas:
            for sgn in (+1, -1):
                q = tuple(p[a] + sgn * dl[a] for a in range(d))
                lower = p if sgn > 0 else q
                w = edges(lower, dl)
                if w == 0.0:
                    continue
                A[i, i] += w
                if q in ids:
                    A[i, ids[q]] -= w
    return A.tocsr()


def _cell_value(arr, d, n, c):
    """Value of a per-cell array (x fastest) at lower corner c, 0 outside."""
    if any(v < 0 or v >= n for v in c):
        return 0.0
    idx = 0
    for a in range(d - 1, -1, -1):
        idx = idx * n + c[a]
    return arr[idx]


@pytest.mark.parametrize("d,n", [(2, 5), (2, 6), (3, 3), (3, 4)])
def test_scalar_coefficient_matches_the_closed_form_edge_weights(d, n):
    rng = np.random.default_rng(11)
    kappa = np.exp(rng.uniform(0.0, 2.0, size=n ** d))
    h = 1.0 / n
    K = lambda c: _cell_value(kappa, d, n, c)   # noqa: E731

    def edges(p, dl):
        if sum(dl) != 1:
            return 0.0
        a = dl.index(1)
        others = [b for b in range(d) if b != a]
        shift = lambda *bs: tuple(p[x] - (1 if x in bs else 0) for x in range(d))   # noqa: E731
        if d == 2:
            return 0.5 * (K(p) + K(shift(others[0])))
        b, c = others
        return h / 6.0 * (2.0 * K(p) + K(shift(b)) + K(shift(c)) + 2.0 * K(shift(b, c)))

    A, _ = assemble_interior(unit_mesh(d, n), W.scalar_coefficient(d, kappa))
    S = _stencil_from_edges(d, n, edges)
    assert abs(A - S).max() < 1e-13 * abs(S).max()
    A1, _ = assemble_interior(unit_mesh(d, n), kappa)     # the kappa-per-cell form of the input
    assert abs(A1 - S).max() < 1e-13 * abs(S).max()


def test_2d_matrix_coefficient_matches_the_closed_form():
    d, n = 2, 6
    rng = np.random.default_rng(12)
    kap = rng.uniform(1.0, 3.0, size=n * n)
    a11, a22 = kap * rng.uniform(0.8, 1.2, size=n * n), kap * rng.uniform(0.8, 1.2, size=n * n)
    a12 = kap * rng.uniform(-0.3, 0.3, size=n * n)
    V = lambda arr, c: _cell_value(arr, d, n, c)   # noqa: E731

    def edges(p, dl):
        if dl == (1, 0):
            below = (p[0], p[1] - 1)
            return 0.5 * ((V(a11, p) - V(a12, p)) + (V(a11, below) - V(a12, below)))
        if dl == (0, 1):
            left = (p[0] - 1, p[1])
            return 0.5 * ((V(a22, p) - V(a12, p)) + (V(a22, left) - V(a12, left)))
        return V(a12, p)            # diagonal (1, 1): both triangles of cell p

    A, _ = assemble_interior(unit_mesh(d, n), np.stack([a11, a12, a22]))
    S = _stencil_from_edges(d, n, edges)
    assert abs(A - S).max() < 1e-13 * abs(S).max()


@pytest.mark.parametrize("d,n", [(2, 6), (3, 4)])
def test_constant_matrix_is_exact_on_quadratics(d, n):
    rng = np.random.default_rng(13)
    G = rng.standard_normal((d, d))
    Am = G @ G.T + d * np.eye(d)
    Hs = rng.standard_normal((d, d))
    Hs = Hs + Hs.T
    bvec = rng.standard_normal(d)
    comps = np.array([[Am[a, b]] * n ** d for a in range(d) for b in range(a, d)])
    mesh = unit_mesh(d, n)
    K, mass = assemble_full(mesh, comps)
    x = mesh.coords
    u = 0.5 * np.einsum("ia,ab,ib->i", x, Hs, x) + x @ bvec + 0.7
    I = mesh.interior
    lhs = (K @ u)[I]
    rhs = -np.trace(Am @ Hs) * mass[I]
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * max(1.0, np.max(np.abs(rhs)))


def _coarse_simplex_of(d, x_local):
    """Kuhn simplex of the unit cell containing local point x: the axis
    order by decreasing coordinate, as a tuple."""
    return tuple(sorted(range(d), key=lambda a: -x_local[a]))


@pytest.mark.parametrize("d,nH,ref", [(2, 2, 2), (3, 2, 1)])
def test_galerkin_levels_are_simplex_means_of_the_finest_matrix(d, nH, ref):
    rng = np.random.default_rng(14)
    n = nH * 2 ** ref
    ncell = n ** d
    comps = W.random_coefficient("r", d, nH, ref, W.F_CUBIC, [3, 3]).coef_cells
    assert comps.shape == (d * (d + 1) // 2, ncell)
    H = Hierarchy(d, nH, ref, coef=comps)
    fine = unit_mesh(d, n)
    At = coefficient_tensors(d, comps)
    for k in range(ref):
        nk = nH * 2 ** k
        cm = unit_mesh(d, nk)
        # volume mean over the fine simplices (all of equal volume) inside each coarse simplex
        acc, cnt = {}, {}
        for simplex in fine.simplices:
            X = fine.coords[simplex]
            cen = X.mean(axis=0)
            low = np.minimum(fine.ijk[simplex].min(axis=0), n - 1)
            cell_f = 0
            for a in range(d - 1, -1, -1):
                cell_f = cell_f * n + int(low[a])
            cc = np.floor(cen * nk).astype(int)
            key = (tuple(cc), _coarse_simplex_of(d, cen * nk - cc))
            acc[key] = acc.get(key, 0.0) + At[cell_f]
            cnt[key] = cnt.get(key, 0) + 1
        assert set(cnt.values()) == {2 ** (d * (ref - k))}
        N = cm.coords.shape[0]
        K = sp.lil_matrix((N, N))
        for simplex in cm.simplices:
            X = cm.coords[simplex]
            cen = X.mean(axis=0)
            cc = np.floor(cen * nk).astype(int)
            key = (tuple(cc), _coarse_simplex_of(d, cen * nk - cc))
            Am = acc[key] / cnt[key]
            M = np.hstack([np.ones((d + 1, 1)), X])
            Cinv = np.linalg.inv(M)
            grads = Cinv[1:, :].T
            vol = abs(np.linalg.det(M)) / math.factorial(d)
            loc = vol * grads @ Am @ grads.T
            for a, i in enumerate(simplex):
                for b, j in enumerate(simplex):
                    K[i, j] += loc[a, b]
        I = cm.interior
        ref_A = K.tocsr()[I][:, I]
        assert abs(H.levels[k].A - ref_A).max() < 1e-12 * abs(ref_A).max()


def test_identity_matrix_gives_the_constant_coefficient_hierarchy():
    d, nH, ref = 3, 2, 2
    n = nH * 2 ** ref
    H0 = Hierarchy(d, nH, ref)
    H1 = Hierarchy(d, nH, ref, coef=W.scalar_coefficient(d, np.ones(n ** d)))
    for a, b in zip(H0.levels, H1.levels):
        assert abs(a.A - b.A).max() < 1e-13 * abs(a.A).max()


@pytest.mark.parametrize("d,n", [(2, 6), (3, 4)])
def test_constant_scaling_symmetry_and_row_sums(d, n):
    mesh = unit_mesh(d, n)
    A1, m1 = assemble_interior(mesh)
    A3, m3 = assemble_interior(mesh, np.full(n ** d, 3.0))
    assert abs(A3 - 3.0 * A1).max() < 1e-14 * abs(A3).max()
    assert np.array_equal(m1, m3)                    # the coefficient leaves the mass alone
    comps = W.random_coefficient("r", d, n, 0, W.F_CUBIC, [4]).coef_cells
    K, _ = assemble_full(mesh, comps)
    assert abs(K - K.T).max() < 1e-14 * abs(K).max()
    assert np.max(np.abs(K @ np.ones(K.shape[0]))) < 1e-13 * abs(K).max()


@pytest.mark.parametrize("d,n", [(2, 12), (3, 5)])
def test_unit_weight_and_zero_weight(d, n):
    rng = np.random.default_rng(15)
    mesh = unit_mesh(d, n)
    g = rng.standard_normal(mesh.coords.shape[0])
    comps = W.random_coefficient("r", d, n, 0, W.F_CUBIC, [5]).coef_cells
    nl = Nonlinearity(W.F_U_PLUS_SIN)
    a = solve_fine(d, n, g, nl, coef=comps)
    b = solve_fine(d, n, g, nl, coef=comps, f_weight=np.ones_like(g))
    assert np.max(np.abs(a.U - b.U)) <= 1e-13 * np.max(np.abs(a.U))
    z = solve_fine(d, n, g, nl, coef=comps, f_weight=np.zeros_like(g))
    A, m = assemble_interior(mesh, comps)
    U = spla.spsolve(A.tocsc(), m * g[mesh.interior])
    assert np.max(np.abs(z.U - U)) <= 1e-12 * np.max(np.abs(U))


@pytest.mark.parametrize("d,n", [(2, 16), (3, 6)])
def test_linear_f_with_weight_is_one_linear_solve(d, n):
    rng = np.random.default_rng(16)
    mesh = unit_mesh(d, n)
    g = rng.standard_normal(mesh.coords.shape[0])
    c = rng.uniform(0.0, 2.0, size=g.size)
    comps = W.random_coefficient("r", d, n, 0, W.F_CUBIC, [6]).coef_cells
    res = solve_fine(d, n, g, Nonlinearity(W.F_LINEAR, 2.5), coef=comps, f_weight=c)
    A, m = assemble_interior(mesh, comps)
    I = mesh.interior
    U = spla.spsolve((A + sp.diags(2.5 * m * c[I])).tocsc(), m * g[I])
    assert np.max(np.abs(res.U - U)) <= 1e-12 * np.max(np.abs(U))


@pytest.mark.parametrize("dim,levels", [(2, (3, 4, 5)), (3, (1, 2, 3))])
@pytest.mark.parametrize("isotropic", [True, False], ids=["kappa", "matrix"])
def test_o1_manufactured_rate_is_second_order(dim, levels, isotropic):
    errs = []
    for L in levels:
        P = W.variable_coefficient("vc", dim, 4, L, W.F_CUBIC if dim == 2 else W.F_U_PLUS_SIN,
                                   isotropic=isotropic)
        r = solve_fine(P.dim, P.n, P.g_nodes, Nonlinearity(P.f_kind), coef=P.coef_cells,
                       f_weight=P.f_weight_nodes)
        errs.append(nodal_l2(r.m, r.U - P.u_exact_nodes[r.mesh.interior]))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(1.85 < q < 2.15 for q in rates), rates


def _problems():
    return [W.variable_coefficient("vc2", 2, 4, 3, W.F_CUBIC),
            W.variable_coefficient("vc3", 3, 4, 2, W.F_U_PLUS_SIN)]


@pytest.mark.parametrize("P", _problems(), ids=["2d", "3d"])
def test_o2_fixed_point_galerkin_and_converged_mode(P):
    nl = Nonlinearity(P.f_kind, P.f_param)
    H = Hierarchy(P.dim, P.coarse_cells, P.refinements, coef=P.coef_cells)
    opts = Options()
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, coef=P.coef_cells, f_weight=P.f_weight_nodes)
    k = H.n_levels - 1
    g_k, c_k = H.g_on_level(P.g_nodes, k), H.g_on_level(P.f_weight_nodes, k)
    u1, _ = correction_step(H, k, o1.U, g_k, nl, opts, None, None, c_k)
    assert np.max(np.abs(u1 - o1.U)) <= 1e-11 * np.max(np.abs(o1.U))
    rng = np.random.default_rng(17)
    ut = o1.U + 1e-2 * rng.standard_normal(o1.U.size)
    z, y, it, ok = augmented_solve(H, k, ut, g_k, nl, opts, None, c_k)
    assert ok
    lev = H.levels[k]
    R = lev.A @ z + lev.m * c_k * nl.f(z) - lev.m * g_k
    B = sp.hstack([lev.Q, sp.csr_matrix(ut.reshape(-1, 1))]).tocsr()
    assert np.max(np.abs(B.T @ R)) < 1e-12 * max(1.0, np.max(np.abs(lev.A @ z)))
    # the coarse block of the augmented matrix is A_1 on every level (one form)
    assert np.max(np.abs((lev.Q.T @ lev.A @ lev.Q).toarray() - H.A1)) < 1e-12 * np.max(np.abs(H.A1))
    res = fmg(H, P.g_nodes, nl, opts, converged=True, f_weight=P.f_weight_nodes)
    assert res.converged_ok
    assert nodal_l2(o1.m, res.U - o1.U) <= 1e-10 * nodal_l2(o1.m, o1.U)


@pytest.mark.parametrize("dim,L", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_o2_meets_the_theorem_3_2_gate(dim, L):
    P = W.variable_coefficient("vc", dim, 4, L, W.F_CUBIC if dim == 2 else W.F_U_PLUS_SIN)
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, coef=P.coef_cells, f_weight=P.f_weight_nodes)
    I = o1.mesh.interior
    disc = nodal_l2(o1.m, o1.U - P.u_exact_nodes[I])
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements, coef=P.coef_cells), P.g_nodes, nl,
              Options(), f_weight=P.f_weight_nodes)
    alg = nodal_l2(o1.m, res.U - o1.U)
    assert alg <= 0.5 * disc, (alg, disc)
    assert nodal_l2(o1.m, res.U - P.u_exact_nodes[I]) <= 1.1 * disc


@pytest.mark.parametrize("dim,nH,L", [(2, 4, 3), (3, 4, 2)])
def test_random_coefficient_converged_mode_reaches_ubar(dim, nH, L):
    """A rough anisotropic coefficient (contrast 10 per cell) and random c:
    no closed-form solution, so the pin is O1's discrete solution."""
    P = W.random_coefficient("rc", dim, nH, L, W.F_U_PLUS_SIN, [5, 1])
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, coef=P.coef_cells, f_weight=P.f_weight_nodes)
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements, coef=P.coef_cells), P.g_nodes, nl,
              Options(), converged=True, f_weight=P.f_weight_nodes)
    assert res.converged_ok
    assert nodal_l2(o1.m, res.U - o1.U) <= 1e-10 * nodal_l2(o1.m, o1.U)


def test_element_rule_with_weight_is_rejected():
    P = W.variable_coefficient("vc", 2, 4, 2, W.F_CUBIC)
    with pytest.raises(ValueError):
        solve_fine(2, P.n, P.g_nodes, Nonlinearity(P.f_kind), quadrature="element", f_weight=P.f_weight_nodes)


@pytest.mark.parametrize("d,n,with_coef", [(2, 6, True), (3, 4, True), (3, 3, False)])
def test_local_rows_equal_the_assembled_rows(d, n, with_coef):
    """local_rows (the rows of a few nodes, for sizes whose whole assembly does
    not fit in memory) against the element-by-element assembly, boundary and
    corner nodes included."""
    mesh = unit_mesh(d, n)
    comps = W.random_coefficient("r", d, n, 0, W.F_CUBIC, [18]).coef_cells if with_coef else None
    K, m = assemble_full(mesh, comps)
    pick = np.concatenate([np.random.default_rng(19).choice(mesh.coords.shape[0], 12, replace=False), [0, mesh.coords.shape[0] - 1]])
    cols, vals, mass = local_rows(d, n, mesh.ijk[pick], comps)
    for k, i in enumerate(pick):
        row = K.getrow(i).toarray().ravel()
        got = np.zeros_like(row)
        got[cols[k]] = vals[k]
        assert np.max(np.abs(got - row)) < 1e-13 * max(1.0, np.max(np.abs(row)))
    assert np.max(np.abs(mass - m[pick])) < 1e-15
