"""Pins of the oracle's element-quadrature reading (oracle/quadrature.py and
the quadrature="element" paths of O1 and O2).

What fixes them, independently of the code under test:
  * the rules integrate every polynomial of degree <= 2 exactly on a simplex:
    the integral of lambda^alpha over a simplex T is |T| d! alpha! / (|alpha| + d)!;
  * for f(u) = c u the rule is exact, so N(u) = c M u with the textbook P1
    element mass matrix M_T = |T| (1 + delta_ij) / ((d+1)(d+2));
  * (g_I, phi_i) for g = 1 is the integral of phi_i, i.e. the lumped mass, and
    the sum over all nodes of (g_I, phi_i) for a linear g is the integral of g;
  * the nonlinear term is the gradient of the energy and the Jacobian its
    derivative (finite differences);
  * a brute-force evaluation on a tiny mesh with explicit loops over
    simplices and points in physical coordinates;
  * O1 for linear f is one sparse linear solve with the textbook mass matrix;
    O1 converges at O(h^2); O2 keeps ubar_h fixed, its augmented step solves
    its Galerkin equations, converged mode reaches ubar_h, and the algebraic
    error stays within half the discretisation error (Theorem 3.2).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fem import assemble_full, assemble_interior, simplex_geometry
from oracle.mesh import unit_mesh
from oracle.nonlinear import Nonlinearity
from oracle.norms import nodal_l2
from oracle.o1 import solve_fine
from oracle.o2 import Hierarchy, Options, augmented_solve, correction_step, fmg
from oracle.quadrature import ElementQuadrature, full_vector, local_element_terms, simplex_rule
from paper_1611_05677_amd import workloads as W


@pytest.mark.parametrize("d", [2, 3])
def test_rule_is_exact_for_degree_two(d):
    pts, w = simplex_rule(d)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(pts.sum(axis=1), 1.0)
    for alpha in itertools.product(range(3), repeat=d + 1):
        if sum(alpha) > 2:
            continue
        q = float(np.sum(w * np.prod(pts ** np.array(alpha), axis=1)))
        exact = math.factorial(d) * np.prod([math.factorial(a) for a in alpha]) / math.factorial(sum(alpha) + d)
        assert abs(q - exact) < 1e-15, (alpha, q, exact)


def _textbook_mass(mesh):
    d = mesh.dim
    _, vol, _ = simplex_geometry(mesh.coords[mesh.simplices])
    loc = np.ones((d + 1, d + 1)) + np.eye(d + 1)
    rows = np.repeat(mesh.simplices, d + 1, axis=1).reshape(-1)
    cols = np.tile(mesh.simplices, (1, d + 1)).reshape(-1)
    vals = (vol[:, None, None] * loc[None] / ((d + 1) * (d + 2))).reshape(-1)
    N = mesh.coords.shape[0]
    M = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    M.sum_duplicates()
    return M


@pytest.mark.parametrize("d,n", [(2, 6), (3, 3)])
def test_linear_f_gives_the_consistent_mass_matrix(d, n):
    mesh = unit_mesh(d, n)
    Qd = ElementQuadrature(mesh)
    M = _textbook_mass(mesh)
    rng = np.random.default_rng(1)
    u = full_vector(mesh, rng.standard_normal(mesh.interior.size))
    nl = Nonlinearity(W.F_LINEAR, 2.5)
    assert np.max(np.abs(Qd.nonlinear(u, nl) - 2.5 * (M @ u))) < 1e-15
    K = Qd.jacobian(u, nl)
    assert abs(K - 2.5 * M).max() < 1e-15
    # energy of c u^2 / 2: c/2 u^T M u
    assert abs(Qd.energy(u, nl) - 1.25 * u @ (M @ u)) < 1e-14


@pytest.mark.parametrize("d,n", [(2, 5), (3, 3)])
def test_load_of_constants_and_linear_functions(d, n):
    mesh = unit_mesh(d, n)
    Qd = ElementQuadrature(mesh)
    _, lumped = assemble_full(mesh)
    assert np.max(np.abs(Qd.load(np.ones(mesh.coords.shape[0])) - lumped)) < 1e-15
    x = mesh.coords
    g = 1.0 + 2.0 * x[:, 0] - 3.0 * x[:, -1]
    exact = 1.0 + 1.0 - 1.5          # integral of g over the unit square / cube
    assert abs(Qd.load(g).sum() - exact) < 1e-13


@pytest.mark.parametrize("kind,param", [(W.F_U_PLUS_SIN, 0.0), (W.F_CUBIC, 0.0), (W.F_NEG_EXP, 0.0),
                                        (W.F_SIGNED_POW, 1.5)])
def test_nonlinear_term_is_the_energy_gradient(kind, param):
    mesh = unit_mesh(2, 4)
    Qd = ElementQuadrature(mesh)
    nl = Nonlinearity(kind, param)
    rng = np.random.default_rng(2)
    u = full_vector(mesh, 0.7 * rng.standard_normal(mesh.interior.size))
    v = full_vector(mesh, rng.standard_normal(mesh.interior.size))
    eps = 1e-5
    fd = (Qd.energy(u + eps * v, nl) - Qd.energy(u - eps * v, nl)) / (2 * eps)
    assert abs(fd - Qd.nonlinear(u, nl) @ v) < 1e-8 * max(1.0, abs(fd))
    fdv = (Qd.nonlinear(u + eps * v, nl) - Qd.nonlinear(u - eps * v, nl)) / (2 * eps)
    assert np.max(np.abs(fdv - Qd.jacobian(u, nl) @ v)) < 1e-7


@pytest.mark.parametrize("d", [2, 3])
def test_brute_force_on_a_tiny_mesh(d):
    """Explicit loops: every simplex, every point (in physical coordinates),
    the P1 interpolant evaluated by solving for barycentric coordinates."""
    n = 2
    mesh = unit_mesh(d, n)
    nl = Nonlinearity(W.F_U_PLUS_SIN)
    rng = np.random.default_rng(3)
    u = full_vector(mesh, rng.standard_normal(mesh.interior.size))
    g = rng.standard_normal(mesh.coords.shape[0])
    pts, w = simplex_rule(d)
    N_ref = np.zeros(mesh.coords.shape[0])
    G_ref = np.zeros(mesh.coords.shape[0])
    for simplex in mesh.simplices:
        V = mesh.coords[simplex]                       # (d+1, d)
        vol = abs(np.linalg.det(V[1:] - V[0])) / math.factorial(d)
        for lam_q, wq in zip(pts, w):
            x = lam_q @ V                              # the point
            # barycentric coordinates of x recovered from the vertices
            Mx = np.vstack([np.ones(d + 1), V.T])
            lam = np.linalg.solve(Mx, np.concatenate([[1.0], x]))
            uq = lam @ u[simplex]
            gq = lam @ g[simplex]
            for a, node in enumerate(simplex):
                N_ref[node] += vol * wq * nl.f(uq) * lam[a]
                G_ref[node] += vol * wq * gq * lam[a]
    Qd = ElementQuadrature(mesh)
    assert np.max(np.abs(Qd.nonlinear(u, nl) - N_ref)) < 1e-15 * 100
    assert np.max(np.abs(Qd.load(g) - G_ref)) < 1e-15 * 100


@pytest.mark.parametrize("d,n", [(2, 16), (3, 6)])
def test_o1_linear_f_is_one_linear_solve(d, n):
    mesh = unit_mesh(d, n)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(mesh.coords.shape[0])
    c = 3.0
    res = solve_fine(d, n, g, Nonlinearity(W.F_LINEAR, c), quadrature="element")
    A, _ = assemble_interior(mesh)
    M = _textbook_mass(mesh)
    I = mesh.interior
    U = spla.spsolve((A + c * M[I][:, I]).tocsc(), (M @ g)[I])
    assert np.max(np.abs(res.U - U)) <= 1e-12 * np.max(np.abs(U))


def test_o1_element_rate_is_second_order():
    errs = []
    for L in (3, 4, 5):
        P = W.square_cubic_sin(L)
        r = solve_fine(P.dim, P.n, P.g_nodes, Nonlinearity(P.f_kind), quadrature="element")
        errs.append(nodal_l2(r.m, r.U - P.u_exact_nodes[r.mesh.interior]))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < q < 2.1 for q in rates), rates


@pytest.mark.parametrize("dim,L", [(2, 3), (3, 2)])
def test_o2_element_fixed_point_galerkin_and_converged_mode(dim, L):
    P = W.square_cubic_sin(L) if dim == 2 else W.cube_u_plus_sin(L)
    nl = Nonlinearity(P.f_kind, P.f_param)
    H = Hierarchy(P.dim, P.coarse_cells, P.refinements)
    opts = Options(quadrature="element")
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, quadrature="element")
    k = H.n_levels - 1
    g_k, gf = H.g_on_level(P.g_nodes, k), H.g_full_on_level(P.g_nodes, k)
    # ubar_h is a fixed point of Algorithm 3.1
    u1, _ = correction_step(H, k, o1.U, g_k, nl, opts, None, gf)
    assert np.max(np.abs(u1 - o1.U)) <= 1e-11 * np.max(np.abs(o1.U))
    # the augmented step solves its Galerkin equations B^T R(z) = 0
    rng = np.random.default_rng(5)
    ut = o1.U + 1e-2 * rng.standard_normal(o1.U.size)
    z, y, it, ok = augmented_solve(H, k, ut, g_k, nl, opts, gf)
    assert ok
    lev = H.levels[k]
    Qd, I = H.quad(k), lev.mesh.interior
    R = lev.A @ z + Qd.nonlinear(full_vector(lev.mesh, z), nl)[I] - Qd.load(gf)[I]
    B = sp.hstack([lev.Q, sp.csr_matrix(ut.reshape(-1, 1))]).tocsr()
    assert np.max(np.abs(B.T @ R)) < 1e-12 * max(1.0, np.max(np.abs(lev.A @ z)))
    # converged mode reaches ubar_h
    res = fmg(H, P.g_nodes, nl, opts, converged=True)
    assert res.converged_ok
    assert nodal_l2(o1.m, res.U - o1.U) <= 1e-10 * nodal_l2(o1.m, o1.U)


@pytest.mark.parametrize("dim,L", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_o2_element_meets_the_theorem_3_2_gate(dim, L):
    P = W.square_cubic_sin(L) if dim == 2 else W.cube_u_plus_sin(L)
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, quadrature="element")
    I = o1.mesh.interior
    disc = nodal_l2(o1.m, o1.U - P.u_exact_nodes[I])
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements), P.g_nodes, nl, Options(quadrature="element"))
    alg = nodal_l2(o1.m, res.U - o1.U)
    assert alg <= 0.5 * disc, (alg, disc)
    assert nodal_l2(o1.m, res.U - P.u_exact_nodes[I]) <= 1.1 * disc


@pytest.mark.parametrize("d,n", [(2, 6), (3, 4)])
def test_local_element_terms_equal_the_whole_mesh_quadrature(d, n):
    """local_element_terms (the element rule at a few nodes, for sizes whose
    whole mesh does not fit in memory) against ElementQuadrature, boundary
    nodes included."""
    mesh = unit_mesh(d, n)
    Qd = ElementQuadrature(mesh)
    nl = Nonlinearity(W.F_U_PLUS_SIN)
    rng = np.random.default_rng(6)
    u = full_vector(mesh, rng.standard_normal(mesh.interior.size))
    g = rng.standard_normal(mesh.coords.shape[0])
    pick = np.concatenate([rng.choice(mesh.coords.shape[0], 12, replace=False), [0]])
    N, G = local_element_terms(d, n, mesh.ijk[pick], u, g, nl)
    assert np.max(np.abs(N - Qd.nonlinear(u, nl)[pick])) < 1e-15 * 100
    assert np.max(np.abs(G - Qd.load(g)[pick])) < 1e-15 * 100
