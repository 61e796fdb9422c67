"""GPU parity of the element-quadrature reading (fmg_options.quadrature =
FMG_QUAD_ELEMENT) through the C ABI.

* paper mode against the oracle's replica O2 with the element rule, element
  by element: relative L2 <= 1e-10 (float64), the mixed-precision bar
  otherwise; Newton counts (level 1 and per level) within one, the
  coefficient of u~ per level to 1e-9;
* converged mode against O1 with the element rule (the exact discrete
  solution of eq. "FEM_form" under this reading): relative L2 <= 1e-10;
* loads that do not vanish on the boundary (the element rule interpolates g
  on boundary simplices too), coarse grids other than 4 cells per side (the
  general Newton paths), graph replay, and the rejected combinations.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from oracle.fem import local_rows  # noqa: E402
from oracle.nonlinear import Nonlinearity  # noqa: E402
from oracle.quadrature import local_element_terms  # noqa: E402
from oracle.norms import nodal_l2  # noqa: E402
from oracle.o1 import solve_fine  # noqa: E402
from oracle.o2 import Hierarchy as O2H  # noqa: E402
from oracle.o2 import Options as O2Options  # noqa: E402
from oracle.o2 import fmg as o2_fmg  # noqa: E402
from paper_1611_05677_amd import binding as B  # noqa: E402
from paper_1611_05677_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
PARITY = 1e-10
MIXED_TOL = 1e-8     # float32 rounding of the corrections (as for the vertex rule)
ELEM = O2Options(quadrature="element")


def gpu_solve(P, **opt):
    H = B.Hierarchy(P.dim, P.coarse_cells, P.refinements,
                    B.default_options(P.dim, quadrature=B.FMG_QUAD_ELEMENT, **opt), device=DEV)
    g = torch.from_numpy(P.g_nodes).to(DEV)
    u, rep = H.solve(g, P.f_kind, P.f_param)
    out = u.cpu().numpy()
    H.close()
    return out, rep


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    W.square_cubic_sin(1), W.square_cubic_sin(3), W.square_cubic_sin(5),
    W.fourier_problem("e_sin", 2, 4, 4, W.F_U_PLUS_SIN, [9, 1]),
    W.fourier_problem("e_abs", 2, 4, 4, W.F_ABS_U_U, [9, 2]),
    W.fourier_problem("e_pow", 2, 4, 3, W.F_SIGNED_POW, [9, 3], f_param=1.5),
    W.fourier_problem("e_lin", 2, 4, 3, W.F_LINEAR, [9, 4], f_param=2.0),
    W.constant_load("e_exp_2d", 2, 4, 4, 1.0, W.F_NEG_EXP),
    W.cube_u_plus_sin(1), W.cube_u_plus_sin(2), W.cube_u_plus_sin(3),
    W.cube_example1(2), W.cube_example3(2), W.cube_example2(2),
    W.fourier_problem("e3_cubic", 3, 4, 2, W.F_CUBIC, [9, 5]),
    # general level-1 and Newton paths (N_1 not 9 or 27)
    W.fourier_problem("e_nH3_2d", 2, 3, 4, W.F_U_PLUS_SIN, [9, 6]),
    W.fourier_problem("e_nH2_3d", 3, 2, 3, W.F_CUBIC, [9, 7]),
]


@pytest.mark.parametrize("P", CASES, ids=[p.name for p in CASES])
def test_element_paper_mode_matches_cpu_replica(P):
    u, rep = gpu_solve(P)
    assert rep["status"] == 0, rep
    res = o2_fmg(O2H(P.dim, P.coarse_cells, P.refinements), P.g_nodes, Nonlinearity(P.f_kind, P.f_param), ELEM)
    expect = res.full()
    assert rel(u, expect) <= PARITY, rel(u, expect)
    assert abs(rep["level1_iters"] - res.level1_iters) <= 1, (rep["level1_iters"], res.level1_iters)
    for s in res.steps:
        assert abs(rep["newton_iters"][s.level - 1] - s.newton_iters) <= 1
        assert abs(rep["alpha"][s.level - 1] - s.alpha) <= 1e-9 * max(1.0, abs(s.alpha))


@pytest.mark.parametrize("P", [W.square_cubic_sin(4), W.cube_u_plus_sin(3), W.constant_load("e_exp_m", 3, 4, 2, 1.0,
                                                                                           W.F_NEG_EXP)],
                         ids=["sq", "cube", "exp3"])
def test_element_mixed_precision_matches_replica(P):
    u, rep = gpu_solve(P, precision=B.FMG_MIXED)
    assert rep["status"] == 0, rep
    expect = o2_fmg(O2H(P.dim, P.coarse_cells, P.refinements), P.g_nodes,
                    Nonlinearity(P.f_kind, P.f_param), ELEM).full()
    assert rel(u, expect) <= MIXED_TOL, rel(u, expect)


@pytest.mark.parametrize("P", [W.square_cubic_sin(4), W.cube_u_plus_sin(2)], ids=["sq", "cube"])
def test_element_converged_mode_matches_fine_newton(P):
    u, rep = gpu_solve(P, mode=B.FMG_CONVERGED)
    assert rep["status"] == 0 and rep["extra_steps"] >= 1, rep
    ref = solve_fine(P.dim, P.n, P.g_nodes, Nonlinearity(P.f_kind, P.f_param), quadrature="element").full()
    assert rel(u, ref) <= PARITY, rel(u, ref)


@pytest.mark.parametrize("P", [W.square_cubic_sin(5), W.cube_u_plus_sin(3)], ids=["sq", "cube"])
def test_element_solution_meets_the_gate_and_differs_from_vertex_rule_at_order_h2(P):
    """Theorem 3.2's gate under the element reading, and the two readings'
    discrete solutions within the discretisation error of each other."""
    u, rep = gpu_solve(P)
    nl = Nonlinearity(P.f_kind, P.f_param)
    o1 = solve_fine(P.dim, P.n, P.g_nodes, nl, quadrature="element")
    I = o1.mesh.interior
    disc = nodal_l2(o1.m, o1.U - P.u_exact_nodes[I])
    assert nodal_l2(o1.m, u[I] - o1.U) <= 0.5 * disc
    assert nodal_l2(o1.m, u[I] - P.u_exact_nodes[I]) <= 1.1 * disc
    H = B.Hierarchy(P.dim, P.coarse_cells, P.refinements, B.default_options(P.dim), device=DEV)
    uv, _ = H.solve(torch.from_numpy(P.g_nodes).to(DEV), P.f_kind, P.f_param)
    H.close()
    assert nodal_l2(o1.m, u[I] - uv.cpu().numpy()[I]) <= 2.0 * disc


def test_element_graph_and_direct_launches_agree_bitwise():
    P = W.cube_u_plus_sin(2)
    a, _ = gpu_solve(P)
    b, _ = gpu_solve(P, use_graph=0)
    assert np.array_equal(a, b)


def test_element_rejects_fused_small_levels():
    with pytest.raises(RuntimeError):
        B.Hierarchy(2, 4, 3, B.default_options(2, quadrature=B.FMG_QUAD_ELEMENT, fuse_small_levels=1), device=DEV)


def test_full_size_element_solution_against_oracle_rows_and_the_gate():
    """The element-rule bench workload at its size (3D 256^3, f = u + sin u),
    whose whole mesh the oracle cannot hold: the oracle forms the discrete
    problem's equations at 512 seeded interior nodes one by one (stiffness
    rows, and the element rule on the simplices around each node) and the
    library's converged-mode solution must satisfy them to 1e-10 of each
    equation's term scale; with it as ubar_h the paper-mode solve meets both
    gate conditions over every node."""
    P = W.cube_u_plus_sin(6)
    n = P.n
    nl = Nonlinearity(P.f_kind, P.f_param)
    g = torch.from_numpy(P.g_nodes).to(DEV)
    H = B.Hierarchy(3, 4, 6, B.default_options(3, quadrature=B.FMG_QUAD_ELEMENT, mode=B.FMG_CONVERGED), device=DEV)
    uct, crep = H.solve(g, P.f_kind, P.f_param)
    H.close()
    assert crep["status"] == 0, crep
    uc = uct.cpu().numpy()
    rng = np.random.default_rng(35)
    ijk = rng.integers(1, n, size=(512, 3))
    cols, vals, _ = local_rows(3, n, ijk)
    N, G = local_element_terms(3, n, ijk, uc, P.g_nodes, nl)
    worst = 0.0
    for k in range(len(ijk)):
        au = vals[k] @ uc[cols[k]]
        scale = np.abs(vals[k]) @ np.abs(uc[cols[k]]) + abs(N[k]) + abs(G[k])
        worst = max(worst, abs(au + N[k] - G[k]) / scale)
    assert worst <= 1e-10, worst
    u, rep = gpu_solve(P)
    assert rep["status"] == 0, rep
    h3 = (1.0 / n) ** 3
    nodal = lambda v: float(np.sqrt(h3 * np.sum(v * v)))   # noqa: E731
    disc = nodal(uc - P.u_exact_nodes)
    assert nodal(u - uc) <= 0.5 * disc
    assert nodal(u - P.u_exact_nodes) <= 1.1 * disc
