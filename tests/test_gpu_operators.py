"""GPU parity of the multigrid-cycle operators against the oracle's
element-assembled CSR stiffness matrices and point-location prolongations.

Each operator is called through the C ABI (fmg_level_op) on random nodal
vectors, at sizes spanning one to several 256-wide tiles plus a ragged tail,
in float64 (bar: 1e-14 relative) and float32 (bar: 2e-6 relative).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from oracle.fem import assemble_full, prolongation  # noqa: E402
from oracle.mesh import unit_mesh  # noqa: E402
from paper_1611_05677_amd import binding as B  # noqa: E402

DEV = "cuda:0"
CASES = [(2, 4, 7), (3, 4, 4)]   # (dim, coarse cells, refinements): 2D up to 512^2, 3D up to 64^3
TOL = {B.FMG_FP64: 1e-14, B.FMG_MIXED: 2e-6}

_H = {}


def hier(dim, nH, L):
    key = (dim, nH, L)
    if key not in _H:
        _H[key] = B.Hierarchy(dim, nH, L, B.default_options(dim, precision=B.FMG_MIXED), device=DEV)
    return _H[key]


def rand_nodes(mesh, seed):
    v = np.random.default_rng(seed).standard_normal(mesh.coords.shape[0])
    v[mesh.boundary] = 0.0
    return v


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def levels_of(dim, L):
    return list(range(1, L + 2)) if dim == 2 else list(range(1, L + 2))


@pytest.mark.parametrize("dim,nH,L", CASES)
@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_apply_A_matches_assembled_stiffness(dim, nH, L, prec):
    H = hier(dim, nH, L)
    for k in levels_of(dim, L):
        mesh = unit_mesh(dim, nH * 2 ** (k - 1))
        K, _ = assemble_full(mesh)
        x = rand_nodes(mesh, k)
        expect = K @ x
        expect[mesh.boundary] = 0.0
        got = H.level_op(B.FMG_OP_APPLY_A, k, to_dev(x), precision=prec).cpu().numpy()
        err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
        assert err < TOL[prec], (k, err)


@pytest.mark.parametrize("dim,nH,L", CASES)
@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_jacobi_sweep(dim, nH, L, prec):
    H = hier(dim, nH, L)
    for k in levels_of(dim, L):
        mesh = unit_mesh(dim, nH * 2 ** (k - 1))
        K, _ = assemble_full(mesh)
        x, b = rand_nodes(mesh, 10 + k), rand_nodes(mesh, 20 + k)
        w = 0.8
        D = K.diagonal()
        expect = x + w * (b - K @ x) / D
        expect[mesh.boundary] = 0.0
        got = H.level_op(B.FMG_OP_SMOOTH, k, to_dev(x), to_dev(b), precision=prec, omega=w).cpu().numpy()
        err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
        assert err < TOL[prec], (k, err)


@pytest.mark.parametrize("dim,nH,L", CASES)
@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_residual_restriction_is_Pt(dim, nH, L, prec):
    H = hier(dim, nH, L)
    for k in levels_of(dim, L)[1:]:
        fine = unit_mesh(dim, nH * 2 ** (k - 1))
        coarse = unit_mesh(dim, nH * 2 ** (k - 2))
        K, _ = assemble_full(fine)
        P = prolongation(coarse, fine)
        x, b = rand_nodes(fine, 30 + k), rand_nodes(fine, 40 + k)
        r = (b - K @ x)[fine.interior]
        expect = np.zeros(coarse.coords.shape[0])
        expect[coarse.interior] = P.T @ r
        got = H.level_op(B.FMG_OP_RESTRICT, k, to_dev(x), to_dev(b), precision=prec).cpu().numpy()
        err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
        assert err < 4 * TOL[prec], (k, err)


def _restriction_weights():
    """P^T stencil of an interior coarse node: the oracle's prolongation on
    the 8^3 / 4^3 pair, column of the coarse node (2, 2, 2), as (fine offset,
    weight) pairs (the stencil is the same at every interior coarse node)."""
    coarse, fine = unit_mesh(3, 4), unit_mesh(3, 8)
    P = prolongation(coarse, fine).tocsc()
    col = int(np.nonzero(coarse.interior == 2 + 5 * (2 + 5 * 2))[0][0])
    rows = P.indices[P.indptr[col]:P.indptr[col + 1]]
    vals = P.data[P.indptr[col]:P.indptr[col + 1]]
    return [(fine.ijk[fine.interior[r]] - 4, v) for r, v in zip(rows, vals)]


@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_residual_restriction_full_size_sampled(prec):
    """3D 384^3 (3 coarse cells, 7 refinements), the size class of the
    plane-marching residual + restriction, with 191 interior coarse nodes per
    axis that fill none of its 30-column strips, 14-row chunks or 39-plane
    chunks evenly: P^T (b - A x) at sampled coarse nodes (the strip, chunk and domain
    edges among them) against the oracle's stiffness rows at the 15 fine nodes
    under each (assembled from the simplices around each node) and its
    prolongation weights."""
    from oracle.fem import local_rows
    nH, L = 3, 7
    n = nH * 2 ** L
    nc = n // 2
    H = hier(3, nH, L)
    k = L + 1
    rng = np.random.default_rng(80 + prec)
    bnd = np.zeros((n + 1,) * 3, dtype=bool)
    bnd[[0, -1]] = bnd[:, [0, -1]] = bnd[:, :, [0, -1]] = True
    bnd = bnd.ravel()
    x = rng.standard_normal((n + 1) ** 3)
    b = rng.standard_normal((n + 1) ** 3)
    x[bnd] = 0.0
    b[bnd] = 0.0
    got = H.level_op(B.FMG_OP_RESTRICT, k, to_dev(x), to_dev(b), precision=prec).cpu().numpy()
    assert np.all(got.reshape((nc + 1,) * 3)[[0, -1]] == 0.0)
    edges = [1, 2, 14, 15, 29, 30, 31, 39, 40, 60, 61, 78, 79, 181, 182, 190, 191]
    pick = np.random.default_rng(3).integers(1, nc, size=(40, 3))
    m = len(edges)
    pick = np.concatenate([pick, np.array([(e, edges[(3 * i) % m], edges[(5 * i + 2) % m])
                                           for i, e in enumerate(edges)])])
    W = _restriction_weights()
    idx = lambda q: int(q[0] + (n + 1) * (q[1] + (n + 1) * q[2]))
    expect, gotv = [], []
    for c in pick:
        total = 0.0
        for off, w in W:
            q = 2 * c + off
            cols, vals, _ = local_rows(3, n, q[None])
            total += w * (b[idx(q)] - vals[0] @ x[cols[0]])
        expect.append(total)
        gotv.append(got[int(c[0] + (nc + 1) * (c[1] + (nc + 1) * c[2]))])
    expect, gotv = np.array(expect), np.array(gotv)
    err = np.max(np.abs(gotv - expect)) / np.max(np.abs(expect))
    assert err < 4 * TOL[prec], err


@pytest.mark.parametrize("dim,nH,L", CASES)
@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_prolongation_is_natural_inclusion(dim, nH, L, prec):
    H = hier(dim, nH, L)
    for k in levels_of(dim, L)[1:]:
        fine = unit_mesh(dim, nH * 2 ** (k - 1))
        coarse = unit_mesh(dim, nH * 2 ** (k - 2))
        P = prolongation(coarse, fine)
        xc, xf = rand_nodes(coarse, 50 + k), rand_nodes(fine, 60 + k)
        expect = xf.copy()
        expect[fine.interior] += P @ xc[coarse.interior]
        got = H.level_op(B.FMG_OP_PROLONG, k, to_dev(xc), to_dev(xf), precision=prec).cpu().numpy()
        err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
        assert err < TOL[prec], (k, err)


@pytest.mark.parametrize("dim,nH,L", CASES)
@pytest.mark.parametrize("prec", [B.FMG_FP64, B.FMG_MIXED])
def test_coarse_solve(dim, nH, L, prec):
    H = hier(dim, nH, L)
    mesh = unit_mesh(dim, nH)
    K, _ = assemble_full(mesh)
    I = mesh.interior
    b = rand_nodes(mesh, 70)
    expect = np.zeros_like(b)
    expect[I] = np.linalg.solve(K[I][:, I].toarray(), b[I])
    got = H.level_op(B.FMG_OP_COARSE, 1, to_dev(b), precision=prec).cpu().numpy()
    err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
    assert err < 10 * TOL[prec], err


def test_level_kernel_timer():
    """fmg_time_level_kernel: positive durations, the stated byte model, and
    a clear error for a kernel variant the options do not select."""
    H = B.Hierarchy(2, 4, 6, B.default_options(2, precision=B.FMG_MIXED), device=DEV)
    N, Nc = (H.n - 1) ** 2, (H.n // 2 - 1) ** 2
    for name, s in (("pre_sweeps_restrict_2d_stream_f64", 8), ("prolong_post_sweeps_2d_stream_f32", 4)):
        ms, nb = B.time_level_kernel(H, name, H.levels, 5)
        assert ms > 0 and nb == s * (3 * N + Nc)
    ms, nb = B.time_level_kernel(H, "smooth_f64", 3, 3)      # level 3: n = 16
    assert ms > 0 and nb == 8 * 3 * 15 ** 2
    with pytest.raises(B.FMGError):
        B.time_level_kernel(H, "pre_sweeps_restrict_2d_f64", H.levels, 1)   # LDS variant not selected
    with pytest.raises(B.FMGError):
        B.time_level_kernel(H, "smooth_f64", 1, 1)                          # level 1 has no sweep
    H.close()
    H3 = B.Hierarchy(3, 4, 3, device=DEV)
    ms, nb = B.time_level_kernel(H3, "smooth_f64", H3.levels, 3)
    assert ms > 0 and nb == 8 * 3 * (H3.n - 1) ** 3
    with pytest.raises(B.FMGError):
        B.time_level_kernel(H3, "smooth_3d_stream_f64", H3.levels, 1)        # not selected by default
    H3s = B.Hierarchy(3, 4, 3, B.default_options(3, sweep_rows=8), device=DEV)
    ms, nb = B.time_level_kernel(H3s, "smooth_3d_stream_f64", H3s.levels, 3)
    assert ms > 0 and nb == 8 * 3 * (H3s.n - 1) ** 3
    H3s.close()
    with pytest.raises(B.FMGError):
        B.time_level_kernel(H3, "smooth_f32", H3.levels, 1)                  # no float32 buffers
    H3.close()
