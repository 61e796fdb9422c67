"""Pins of the oracle's variable-coefficient reading: -div(kappa grad u) +
c(x) f(u) = g, kappa > 0 constant on every cell of the finest mesh, c >= 0 at
its nodes (oracle/fem.py, the kappa / f_weight paths of O1 and O2).

What fixes them, independently of the code under test:
  * on the Kuhn split every P1 stiffness entry between two nodes that are not
    the ends of one axis edge vanishes (the split's simplices are orthoschemes:
    the gradients of the barycentric coordinates of non-consecutive path
    vertices are orthogonal), and an axis edge from node p to p + e_a takes
    -h^(d-2) / d! from every simplex in which it is a path step.  Counting the
    simplices gives the edge weight in closed form: in 2D (kappa of the two
    cells beside the edge) / 2; in 3D (2 kappa(p) + kappa(p - e_b) +
    kappa(p - e_c) + 2 kappa(p - e_b - e_c)) h / 6 over the cells named by
    their lower corners, b and c the other two axes.  A brute-force stencil
    built from these weights must equal the element-by-element assembly;
  * kappa = const scales A; A is symmetric with zero row sums before the
    boundary is eliminated;
  * the coarse-level coefficients are means over the 2^d children (explicit
    loops), so a kappa constant on coarse cells reaches every level exactly;
  * c = 1 is the constant-coefficient problem; c = 0 and linear f reduce O1
    to one sparse linear solve with the vertex-rule mass;
  * the manufactured smooth problem converges at O(h^2); O2 keeps ubar_h
    fixed and meets the Theorem 3.2 gate with the coefficients.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fem import assemble_full, assemble_interior
from oracle.mesh import unit_mesh
from oracle.nonlinear import Nonlinearity
from oracle.norms import nodal_l2
from oracle.o1 import solve_fine
from oracle.o2 import Hierarchy, Options, augmented_solve, correction_step, fmg, level_kappas
from paper_1611_05677_amd import workloads as W


def _stencil_matrix(d, n, kappa):
    """Interior stiffness from the closed-form edge weights (explicit loops)."""
    h = 1.0 / n
    kap = np.asarray(kappa).reshape((n,) * d)          # axes (z,) y, x

    def K(c):                                        # c = lower corner (x, y[, z])
        return kap[tuple(reversed(c))]

    def weight(p, a):
        """Edge from node p (x, y[, z]) to p + e_a."""
        others = [b for b in range(d) if b != a]
        if d == 2:
            b = others[0]
            q = list(p)
            q[b] -= 1
            return 0.5 * (K(p) + K(q))
        b, c = others
        pb, pc, pbc = list(p), list(p), list(p)
        pb[b] -= 1
        pc[c] -= 1
        pbc[b] -= 1
        pbc[c] -= 1
        return h / 6.0 * (2.0 * K(p) + K(pb) + K(pc) + 2.0 * K(pbc))

    interior = [p for p in np.ndindex(*((n + 1,) * d)) if all(0 < v < n for v in p)]
    # ndindex runs the first index slowest; node ids are x fastest
    interior = [tuple(reversed(p)) for p in interior]
    ids = {p: i for i, p in enumerate(sorted(interior, key=lambda p: tuple(reversed(p))))}
    A = sp.lil_matrix((len(ids), len(ids)))
    for p, i in ids.items():
        for a in range(d):
            for sgn in (+1, -1):
                q = list(p)
                q[a] += sgn
                lower = tuple(p) if sgn > 0 else tuple(q)
                w = weight(lower, a)
                A[i, i] += w
                if tuple(q) in ids:
                    A[i, ids[tuple(q)]] -= w
    return A.tocsr()


@pytest.mark.parametrize("d,n", [(2, 5), (2, 6), (3, 3), (3, 4)])
def test_assembly_matches_the_closed_form_edge_weights(d, n):
    rng = np.random.default_rng(11)
    kappa = np.exp(rng.uniform(0.0, 2.0, size=n ** d))
    A, _ = assemble_interior(unit_mesh(d, n), kappa)
    S = _stencil_matrix(d, n, kappa)
    assert abs(A - S).max() < 1e-13 * abs(S).max()


@pytest.mark.parametrize("d,n", [(2, 6), (3, 4)])
def test_constant_scaling_symmetry_and_row_sums(d, n):
    mesh = unit_mesh(d, n)
    A1, m1 = assemble_interior(mesh)
    A3, m3 = assemble_interior(mesh, np.full(n ** d, 3.0))
    assert abs(A3 - 3.0 * A1).max() < 1e-14 * abs(A3).max()
    assert np.array_equal(m1, m3)                    # kappa leaves the mass alone
    rng = np.random.default_rng(12)
    kappa = rng.uniform(0.5, 4.0, size=n ** d)
    K, _ = assemble_full(mesh, kappa)
    assert abs(K - K.T).max() < 1e-14 * abs(K).max()
    assert np.max(np.abs(K @ np.ones(K.shape[0]))) < 1e-13 * abs(K).max()


def test_coarse_coefficients_are_child_means():
    d, nH, ref = 2, 3, 2
    n = nH * 2 ** ref
    rng = np.random.default_rng(13)
    kappa = rng.uniform(1.0, 5.0, size=n ** d)
    levels = level_kappas(d, n, ref, kappa)
    assert [lv.size for lv in levels] == [(nH * 2 ** k) ** d for k in range(ref + 1)]
    assert np.array_equal(levels[-1], kappa)
    for k in range(ref):
        nc, nf = nH * 2 ** k, nH * 2 ** (k + 1)
        fine = levels[k + 1]
        for cy in range(nc):
            for cx in range(nc):
                kids = [fine[(2 * cx + ox) + nf * (2 * cy + oy)] for oy in (0, 1) for ox in (0, 1)]
                assert abs(levels[k][cx + nc * cy] - sum(kids) / 4.0) < 1e-15 * 5.0


def test_coefficient_constant_on_coarse_cells_reaches_every_level():
    d, nH, ref = 3, 2, 2
    n = nH * 2 ** ref
    rng = np.random.default_rng(14)
    coarse = rng.uniform(1.0, 5.0, size=(nH,) * d)
    fine = np.kron(coarse, np.ones((2 ** ref,) * d)).reshape(-1)
    H = Hierarchy(d, nH, ref, kappa=fine)
    for k in range(ref + 1):
        s = 2 ** k
        kap_k = np.kron(coarse, np.ones((s,) * d)).reshape(-1)
        A, _ = assemble_interior(unit_mesh(d, nH * s), kap_k)
        assert abs(H.levels[k].A - A).max() < 1e-13 * abs(A).max()


@pytest.mark.parametrize("d,n", [(2, 12), (3, 5)])
def test_unit_weight_and_zero_weight(d, n):
    rng = np.random.default_rng(15)
    mesh = unit_mesh(d, n)
    g = rng.standard_normal(mesh.coords.shape[0])
    kappa = rng.uniform(1.0, 3.0, size=n ** d)
    nl = Nonlinearity(W.F_U_PLUS_SIN)
    a = solve_fine(d, n, g, nl, kappa=kappa)
    b = solve_fine(d, n, g, nl, kappa=kappa, f_weight=np.ones_like(g))
    assert np.max(np.abs(a.U - b.U)) <= 1e-13 * np.max(np.abs(a.U))
    # c = 0: A U = m g
    z = solve_fine(d, n, g, nl, kappa=kappa, f_weight=np.zeros_like(g))
    A, m = assemble_interior(mesh, kappa)
    U = spla.spsolve(A.tocsc(), m * g[mesh.interior])
    assert np.max(np.abs(z.U - U)) <= 1e-12 * np.max(np.abs(U))


@pytest.mark.parametrize("d,n", [(2, 16), (3, 6)])
def test_linear_f_with_weight_is_one_linear_solve(d, n):
    rng = np.random.default_rng(16)
    mesh = unit_mesh(d, n)
    g = rng.standard_normal(mesh.coords.shape[0])
    c = rng.uniform(0.0, 2.0, size=g.size)
    kappa = rng.uniform(1.0, 3.0, size=n ** d)
    res = solve_fine(d, n, g, Nonlinearity(W.F_LINEAR, 2.5), kappa=kappa, f_weight=c)
    A, m = assemble_interior(mesh, kappa)
    I = mesh.interior
    U = spla.spsolve((A + sp.diags(2.5 * m * c[I])).tocsc(), m * g[I])
    assert np.max(np.abs(res.U - U)) <= 1e-12 * np.max(np.abs(U))


@pytest.mark.parametrize("dim,levels", [(2, (3, 4, 5)), (3, (1, 2, 3))])
def test_o1_manufactured_rate_is_second_order(dim, levels):
    errs = []
    for L in levels:
        P = W.variable_coefficient("vc", dim, 4, L, W.F_CUBIC if dim == 2 else W.F_U_PLUS_SIN)
        r = solve_fine(P.dim, P.n, P.g_nodes, Nonlinearity(P.f_kind), kappa=P.kappa_cells,
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
    H = Hierarchy(P.dim, P.coarse_cells, P.refinements, kappa=P.kappa_cells)
    opts = Options()
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, kappa=P.kappa_cells, f_weight=P.f_weight_nodes)
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
    res = fmg(H, P.g_nodes, nl, opts, converged=True, f_weight=P.f_weight_nodes)
    assert res.converged_ok
    assert nodal_l2(o1.m, res.U - o1.U) <= 1e-10 * nodal_l2(o1.m, o1.U)


@pytest.mark.parametrize("dim,L", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_o2_meets_the_theorem_3_2_gate(dim, L):
    P = W.variable_coefficient("vc", dim, 4, L, W.F_CUBIC if dim == 2 else W.F_U_PLUS_SIN)
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, kappa=P.kappa_cells, f_weight=P.f_weight_nodes)
    I = o1.mesh.interior
    disc = nodal_l2(o1.m, o1.U - P.u_exact_nodes[I])
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements, kappa=P.kappa_cells), P.g_nodes, nl,
              Options(), f_weight=P.f_weight_nodes)
    alg = nodal_l2(o1.m, res.U - o1.U)
    assert alg <= 0.5 * disc, (alg, disc)
    assert nodal_l2(o1.m, res.U - P.u_exact_nodes[I]) <= 1.1 * disc


def test_random_coefficient_converged_mode_reaches_ubar():
    """A rough coefficient (log-uniform contrast 10 per cell) and random c:
    no closed-form solution, so the pin is O1's discrete solution."""
    P = W.random_coefficient("rc", 2, 4, 3, W.F_U_PLUS_SIN, [5, 1])
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, kappa=P.kappa_cells, f_weight=P.f_weight_nodes)
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements, kappa=P.kappa_cells), P.g_nodes, nl,
              Options(), converged=True, f_weight=P.f_weight_nodes)
    assert res.converged_ok
    assert nodal_l2(o1.m, res.U - o1.U) <= 1e-10 * nodal_l2(o1.m, o1.U)


def test_element_rule_with_weight_is_rejected():
    P = W.variable_coefficient("vc", 2, 4, 2, W.F_CUBIC)
    with pytest.raises(ValueError):
        solve_fine(2, P.n, P.g_nodes, Nonlinearity(P.f_kind), quadrature="element", f_weight=P.f_weight_nodes)
