"""fmg_solve_noalloc (the entry point for callers that cannot allocate) against
the hierarchy entry points (fmg_create_hierarchy + fmg_solve) on the same
inputs: float64 to 1e-10 relative L2 and mixed precision to 1e-8 (the two
paths run the small levels' V-cycle as a dense operator and as a recursive
single-workgroup cycle, equal up to rounding), on consecutive calls where the
second is smaller than the first (the static scratch keeps the previous
call's contents), plus the size and mode limits."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1611_05677_amd import binding as B  # noqa: E402
from paper_1611_05677_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def hierarchy_solve(P, **opt):
    H = B.Hierarchy(P.dim, P.coarse_cells, P.refinements, B.default_options(P.dim, **opt), device=DEV)
    u, rep = H.solve(torch.from_numpy(P.g_nodes).to(DEV), P.f_kind, P.f_param)
    out = u.cpu().numpy()
    H.close()
    return out, rep


def noalloc_solve(P, **opt):
    g = torch.from_numpy(P.g_nodes).to(DEV)
    rep = torch.zeros(ctypes.sizeof(B.Report), dtype=torch.uint8, device=DEV)
    u = B.solve_noalloc(P.dim, P.coarse_cells, P.refinements, g, P.f_kind, P.f_param,
                        B.default_options(P.dim, **opt), report=rep)
    torch.cuda.synchronize()
    return u.cpu().numpy(), B.report_from_device(rep)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SEQUENCES = [
    # (first, second): the second call is smaller than the first
    ("2d_fp64", [W.square_cubic_sin_expx(8), W.fourier_problem("s2", 2, 4, 5, W.F_ABS_U_U, [5, 1])],
     B.FMG_FP64),
    ("2d_mixed", [W.square_cubic_sin_expx(8), W.square_cubic_sin(4)], B.FMG_MIXED),
    ("3d_fp64", [W.cube_u_plus_sin(4), W.cube_example3(2)], B.FMG_FP64),
    ("3d_mixed", [W.cube_u_plus_sin(4), W.fourier_problem("s3", 3, 4, 3, W.F_CUBIC, [5, 2])], B.FMG_MIXED),
    ("coarse_grids", [W.fourier_problem("c8", 2, 8, 6, W.F_CUBIC, [5, 3]),
                      W.fourier_problem("c3", 3, 3, 3, W.F_U_PLUS_SIN, [5, 4])], B.FMG_FP64),
]


@pytest.mark.parametrize("name,problems,precision", SEQUENCES, ids=[s[0] for s in SEQUENCES])
def test_noalloc_matches_hierarchy_path_on_consecutive_calls(name, problems, precision):
    tol = 1e-10 if precision == B.FMG_FP64 else 1e-8
    first = problems[0]
    assert problems[1].interior_dofs < first.interior_dofs or problems[1].dim != first.dim
    for P in problems:
        u, rep = noalloc_solve(P, precision=precision)
        ref, rep_ref = hierarchy_solve(P, precision=precision)
        assert rep["status"] == 0, rep
        assert rep["levels"] == P.n_levels
        assert rel(u, ref) <= tol, (P.name, rel(u, ref))
        assert all(abs(a - b) <= 1 for a, b in zip(rep["newton_iters"], rep_ref["newton_iters"]))


def test_noalloc_repeats_bitwise():
    P = W.square_cubic_sin_expx(6)
    a, _ = noalloc_solve(P)
    noalloc_solve(W.cube_u_plus_sin(3))      # something else in between
    b, _ = noalloc_solve(P)
    assert np.array_equal(a, b)


def test_noalloc_limits():
    g = torch.zeros((4 * 2 ** 9 + 1) ** 2, dtype=torch.float64, device=DEV)
    with pytest.raises(B.FMGError) as e:           # 2048^2 needs more than the scratch
        B.solve_noalloc(2, 4, 9, g, W.F_CUBIC)
    assert e.value.code == B.FMG_E_SCRATCH
    g = torch.zeros((4 * 2 ** 3 + 1) ** 2, dtype=torch.float64, device=DEV)
    with pytest.raises(B.FMGError) as e:
        B.solve_noalloc(2, 4, 3, g, W.F_CUBIC, opts=B.default_options(2, mode=B.FMG_CONVERGED))
    assert e.value.code == B.FMG_E_UNSUPPORTED
