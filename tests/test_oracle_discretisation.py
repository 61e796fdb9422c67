"""Pins for the oracle's discretisation (mesh, P1 assembly, lumped mass,
transfers, nonlinearity catalogue) against closed forms that the mathematics
fixes, independent of the oracle's own code paths.

Section 2 (eq. "linear_fe_space", eq. "FEM_form"), Section 3 (eq.
"mesh_size_recur", eq. "FEM_Space_Series").
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.fem import assemble_full, assemble_interior, prolongation, simplex_geometry
from oracle.mesh import unit_mesh
from oracle.nonlinear import Nonlinearity
from oracle.o2 import chebyshev_weights
from paper_1611_05677_amd import workloads as W


@pytest.mark.parametrize("d,n", [(2, 4), (2, 7), (3, 4), (3, 5)])
def test_mesh_volumes_and_counts(d, n):
    mesh = unit_mesh(d, n)
    assert mesh.simplices.shape == (math.factorial(d) * n ** d, d + 1)
    _, vol, _ = simplex_geometry(mesh.coords[mesh.simplices])
    np.testing.assert_allclose(vol, (1.0 / n) ** d / math.factorial(d), rtol=1e-12)
    assert abs(vol.sum() - 1.0) < 1e-12
    # conforming: every interior facet is shared by exactly two simplices
    facets = {}
    for s in mesh.simplices:
        for drop in range(d + 1):
            key = tuple(sorted(np.delete(s, drop)))
            facets[key] = facets.get(key, 0) + 1
    counts = np.array(list(facets.values()))
    assert set(counts.tolist()) <= {1, 2}
    # boundary facets: 2 d n^{d-1} (d-1)! of them
    assert (counts == 1).sum() == 2 * d * n ** (d - 1) * math.factorial(d - 1)


def _grid_neighbours(mesh, j):
    ijk = mesh.ijk[j]
    out = []
    for a in range(mesh.dim):
        for s in (-1, 1):
            q = ijk.copy()
            q[a] += s
            idx = 0
            for b in range(mesh.dim - 1, -1, -1):
                idx = idx * (mesh.n + 1) + q[b]
            out.append(idx)
    return out


@pytest.mark.parametrize("d,n", [(2, 4), (2, 8), (3, 4), (3, 6)])
def test_stiffness_stencil_closed_form(d, n):
    """Interior rows are h^{d-2} [2d; -1 on the 2d axis neighbours], all other
    couplings (the Kuhn diagonals) cancel to zero."""
    mesh = unit_mesh(d, n)
    K, mass = assemble_full(mesh)
    K = K.toarray()
    h = 1.0 / n
    scale = h ** (d - 2)
    for j in mesh.interior:
        row = K[j].copy()
        assert abs(row[j] - 2 * d * scale) < 1e-13
        for q in _grid_neighbours(mesh, j):
            assert abs(row[q] + scale) < 1e-13
            row[q] = 0.0
        row[j] = 0.0
        assert np.max(np.abs(row)) < 1e-13
    np.testing.assert_allclose(K, K.T, atol=1e-15)
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-13)      # constants in the kernel
    x = mesh.coords
    for a in range(d):                                               # affine functions
        np.testing.assert_allclose((K @ x[:, a])[mesh.interior], 0.0, atol=1e-13)
    q = (x ** 2).sum(1)                                              # -Laplace(q) = -2d
    np.testing.assert_allclose((K @ q)[mesh.interior], -2 * d * h ** d, atol=1e-13)
    np.testing.assert_allclose(mass[mesh.interior], h ** d, rtol=1e-12)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_sine_modes_are_eigenvectors(d, n):
    """A s_k = h^{d-2} (2d - 2 sum_i cos(k_i pi h)) s_k for the discrete sine modes."""
    mesh = unit_mesh(d, n)
    A, m = assemble_interior(mesh)
    h = 1.0 / n
    X = mesh.coords[mesh.interior]
    rng = np.random.default_rng(0)
    for _ in range(5):
        k = rng.integers(1, n, size=d)
        s = np.prod(np.sin(np.pi * k[None, :] * X), axis=1)
        lam = h ** (d - 2) * (2 * d - 2 * np.sum(np.cos(k * np.pi * h)))
        np.testing.assert_allclose(A @ s, lam * s, atol=1e-12)


@pytest.mark.parametrize("d,nc", [(2, 2), (2, 4), (2, 8), (3, 2), (3, 4)])
def test_prolongation_natural_inclusion(d, nc):
    """P_k is the natural inclusion of nested P1 spaces: entries are 1 (coarse
    node) or 1/2 (midpoint of a coarse edge); P^T A_k P = A_{k-1} (Galerkin
    identity of nested conforming spaces); P^T 1 = 2^d."""
    coarse, fine = unit_mesh(d, nc), unit_mesh(d, 2 * nc)
    Ac, _ = assemble_interior(coarse)
    Af, _ = assemble_interior(fine)
    P = prolongation(coarse, fine)
    vals = np.unique(np.round(P.data, 14))
    assert set(vals.tolist()) <= {0.5, 1.0}
    np.testing.assert_allclose((P.T @ Af @ P).toarray(), Ac.toarray(), atol=1e-13)
    np.testing.assert_allclose(P.T @ np.ones(P.shape[0]), 2.0 ** d, atol=1e-13)
    # each coarse interior node is copied to the coincident fine node
    fpos = {tuple(c): i for i, c in enumerate(fine.ijk[fine.interior])}
    Pd = P.toarray()
    for c, node in enumerate(coarse.interior):
        i = fpos[tuple(2 * coarse.ijk[node])]
        assert Pd[i, c] == 1.0 and np.count_nonzero(Pd[i]) == 1
    # column c has 1 + 2 (2^d - 1) nonzeros: itself and the midpoints of its
    # 2(2^d - 1) Kuhn edges
    nnz = np.count_nonzero(Pd, axis=0)
    assert np.all(nnz == 1 + 2 * (2 ** d - 1))


@pytest.mark.parametrize("kind,param", [(W.F_ZERO, 0), (W.F_LINEAR, 2.5), (W.F_CUBIC, 0),
                                        (W.F_U_PLUS_SIN, 0), (W.F_ABS_U_U, 0),
                                        (W.F_SIGNED_POW, 1.5), (W.F_NEG_EXP, 0)])
def test_nonlinearity_derivatives_and_monotone(kind, param):
    nl = Nonlinearity(kind, param)
    u = np.linspace(-2.3, 2.1, 401)
    u = u[np.abs(u) > 1e-3]
    eps = 1e-6
    fd = (nl.f(u + eps) - nl.f(u - eps)) / (2 * eps)
    np.testing.assert_allclose(nl.df(u), fd, rtol=1e-6, atol=1e-8)
    Fd = (nl.F(u + eps) - nl.F(u - eps)) / (2 * eps)
    np.testing.assert_allclose(Fd, nl.f(u), rtol=1e-6, atol=1e-8)
    assert np.all(nl.df(u) >= 0)
    assert abs(float(nl.F(np.zeros(1))[0])) < 1e-15


def test_chebyshev_weights_equioscillate():
    """p(l) = prod(1 - w_i l) is the scaled Chebyshev polynomial on [1/3, 2]:
    |p| takes its maximum with alternating signs at nu+1 points."""
    for nu in (1, 2, 3, 4):
        w = chebyshev_weights(nu, 1.0 / 3.0, 2.0)
        lam = np.linspace(1.0 / 3.0, 2.0, 20001)
        p = np.prod([1 - wi * lam for wi in w], axis=0)
        pmax = np.max(np.abs(p))
        ext = 0.5 * (2 + 1 / 3) - 0.5 * (2 - 1 / 3) * np.cos(np.pi * np.arange(nu + 1) / nu)
        pe = np.prod([1 - wi * ext for wi in w], axis=0)
        np.testing.assert_allclose(np.abs(pe), pmax, rtol=1e-6)
        assert np.all(np.sign(pe[1:]) != np.sign(pe[:-1]))
    np.testing.assert_allclose(chebyshev_weights(2, 1 / 3, 2), [0.5695013, 1.7318686], atol=1e-7)


def test_fourier_load_matches_direct_sum():
    """The separable evaluation of the random sine-series load equals the plain sum."""
    for d, n in ((2, 8), (3, 4)):
        coef = W.fourier_coefficients(d, 3, [1, 2])
        g = W.fourier_load_nodes(coef, n)
        mesh = unit_mesh(d, n)
        direct = np.zeros(mesh.coords.shape[0])
        for k in np.ndindex(*coef.shape):
            direct += coef[k] * np.prod(np.sin(np.pi * (np.array(k) + 1) * mesh.coords), axis=1)
        np.testing.assert_allclose(g, direct, atol=1e-13)


def test_manufactured_loads_satisfy_pde():
    """g - f(u) equals -Laplace(u) by finite differences of the closed-form u."""
    for P in (W.square_cubic_sin(2), W.square_cubic_sin_expx(2), W.cube_u_plus_sin(1),
              W.cube_example3(1)):
        nl = Nonlinearity(P.f_kind, P.f_param)
        rng = np.random.default_rng(3)
        eps = 1e-4
        mesh = unit_mesh(P.dim, P.n)
        idx = rng.integers(0, mesh.coords.shape[0], size=50)
        idx = idx[~mesh.boundary[idx]]
        X = mesh.coords[idx]
        lapn = np.zeros(idx.size)
        for a in range(P.dim):
            e = np.zeros(P.dim)
            e[a] = eps
            lapn += (P.u_exact(*(X + e).T) - 2 * P.u_exact(*X.T) + P.u_exact(*(X - e).T)) / eps ** 2
        g_minus_f = P.g_nodes[idx] - nl.f(P.u_exact_nodes[idx])
        np.testing.assert_allclose(g_minus_f, -lapn, rtol=1e-5, atol=1e-5)
