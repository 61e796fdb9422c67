"""Pins of the oracle's paper-mode contract and of its converged-mode stop.

The paper fixes m = 2 and p = 1 (Section 4) but leaves the multigrid cycle,
smoother and weights to the reader; the readings taken (V(2,2) cycles, damped
Jacobi 4/5 in 2D, degree-2 Chebyshev weights on [1/3, 2] in 3D, exact level-1
solve, vertex quadrature, H = 1/4) decide the algebraic error of Algorithm 3.2
at the level of its leading digits.  These tests pin that contract to values
measured independently of this oracle, in separate throwaway scripts written
while the method was being surveyed, before any of this code existed:
discretisation error disc = ||I_h u - ubar_h|| and algebraic error
alg = ||u_FMG - ubar_h|| in the nodal norm (h^d sum v^2)^{1/2}.  disc is a
property of the discrete problem (4 digits); alg depends on the whole cycle
contract (3 digits).  A changed default (m, nu, a weight, the smoother, the
Newton start) moves alg by far more than that.

Second, the converged mode: an iteration whose update stops shrinking while
still far from the tolerance (here a divergent smoother weight) must be
reported as not converged; the default iteration reaches the tolerance.
"""
import numpy as np
import pytest

from oracle.nonlinear import Nonlinearity
from oracle.norms import nodal_l2
from oracle.o1 import solve_fine
from oracle.o2 import Hierarchy, Options, fmg
from paper_1611_05677_amd import workloads as W

# (problem, smoother options, disc, alg): survey-time probe values
PROBES = [
    ("sq_sin_n32", lambda: W.square_cubic_sin(3), {}, 3.702e-04, 4.101e-05),
    ("sq_sin_n128", lambda: W.square_cubic_sin(5), {}, 2.313e-05, 2.823e-06),
    ("sq_expx_n128", lambda: W.square_cubic_sin_expx(5), {}, 2.823e-05, 6.038e-06),
    ("sq_usin_n128", lambda: W.manufactured("sq_usin", 2, 4, 5, "sin", W.F_U_PLUS_SIN), {},
     2.307e-05, 2.394e-06),
    ("cube_cheb_n16", lambda: W.cube_u_plus_sin(2), {}, 1.073e-03, 1.006e-04),
    ("cube_cheb_n32", lambda: W.cube_u_plus_sin(3), {}, 2.678e-04, 2.925e-05),
    ("cube_jacobi_n32", lambda: W.cube_u_plus_sin(3), {"smoother": 1}, 2.678e-04, 1.880e-04),
]


def _digits(value, ref, digits):
    return abs(value - ref) <= 0.5 * 10.0 ** (np.floor(np.log10(abs(ref))) - digits + 1) * 1.0001


@pytest.mark.parametrize("name,factory,opts,disc_ref,alg_ref", PROBES, ids=[p[0] for p in PROBES])
def test_paper_mode_reproduces_probe_errors(name, factory, opts, disc_ref, alg_ref):
    P = factory()
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl)
    I = o1.mesh.interior
    disc = nodal_l2(o1.m, o1.U - P.u_exact_nodes[I])
    res = fmg(Hierarchy(P.dim, P.coarse_cells, P.refinements), P.g_nodes, nl, Options(**opts))
    alg = nodal_l2(o1.m, res.U - o1.U)
    assert _digits(disc, disc_ref, 4), (disc, disc_ref)
    assert _digits(alg, alg_ref, 3), (alg, alg_ref)


def test_probe_check_fails_for_a_changed_contract():
    """The 3-digit check of alg is sharp enough to see a one-cycle change."""
    P = W.square_cubic_sin(3)
    nl = Nonlinearity(P.f_kind)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl)
    res = fmg(Hierarchy(2, 4, 3), P.g_nodes, nl, Options(m_vcycles=1))
    assert not _digits(nodal_l2(o1.m, res.U - o1.U), 4.101e-05, 3)
    res = fmg(Hierarchy(2, 4, 3), P.g_nodes, nl, Options(nu_pre=1, nu_post=1))
    assert not _digits(nodal_l2(o1.m, res.U - o1.U), 4.101e-05, 3)


def test_converged_mode_reports_stagnation_far_from_tolerance():
    P = W.square_cubic_sin(3)
    H = Hierarchy(2, 4, 3)
    bad = fmg(H, P.g_nodes, Nonlinearity(P.f_kind), Options(omega=1.9, m_vcycles=1), converged=True)
    assert bad.extra_steps < 40 and bad.last_update_rel > 1e-6
    assert not bad.converged_ok
    good = fmg(H, P.g_nodes, Nonlinearity(P.f_kind), converged=True)
    assert good.converged_ok and good.last_update_rel <= 1e3 * Options().converged_tol


def test_converged_mode_step_cap_is_not_convergence():
    P = W.square_cubic_sin(3)
    res = fmg(Hierarchy(2, 4, 3), P.g_nodes, Nonlinearity(P.f_kind),
              Options(converged_max_steps=2), converged=True)
    assert res.extra_steps == 2 and not res.converged_ok
