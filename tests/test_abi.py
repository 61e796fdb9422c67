"""C ABI checks that need no GPU: the library loads, exports every function
include/fmg.h declares, the ctypes mirrors match the C struct layouts, and
host-side argument validation returns the documented status codes before any
device work is enqueued."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmg.h")

B = pytest.importorskip("paper_1611_05677_amd.binding")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmg_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "fmg_solve" in names and "fmg_create_hierarchy" in names
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fmg_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(B.LIB, n)


def test_struct_layouts_match_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
#define P(T, F) printf(#T "." #F " %zu\\n", offsetof(T, F))
int main(void) {{
  printf("fmg_options %zu\\nfmg_report %zu\\nfmg_problem %zu\\nfmg_mesh_desc %zu\\n",
         sizeof(fmg_options), sizeof(fmg_report), sizeof(fmg_problem), sizeof(fmg_mesh_desc));
  P(fmg_options, omega); P(fmg_options, newton_tol); P(fmg_options, newton_passes);
  P(fmg_options, converged_tol); P(fmg_options, use_graph);
  P(fmg_report, newton_iters); P(fmg_report, newton_total); P(fmg_report, alpha);
  P(fmg_report, last_update_rel); P(fmg_problem, g_nodes); P(fmg_problem, f_weight);
  P(fmg_options, quadrature); P(fmg_options, coefficients);
  return 0;
}}""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(prog)], check=True)
    lines = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                          text=True).stdout.splitlines())
    assert int(lines["fmg_options"]) == ctypes.sizeof(B.Options)
    assert int(lines["fmg_report"]) == ctypes.sizeof(B.Report)
    assert int(lines["fmg_problem"]) == ctypes.sizeof(B.ProblemC)
    assert int(lines["fmg_mesh_desc"]) == ctypes.sizeof(B.MeshDesc)
    for key, val in lines.items():
        if "." in key:
            sname, field = key.split(".")
            cls = {"fmg_options": B.Options, "fmg_report": B.Report, "fmg_problem": B.ProblemC}[sname]
            assert getattr(cls, field).offset == int(val), key


def test_default_options():
    for dim in (2, 3):
        o = B.default_options(dim)
        assert (o.m_vcycles, o.p_steps, o.nu_pre, o.nu_post) == (2, 1, 2, 2)
        assert o.newton_max == 30 and o.newton_tol == 1e-14
        assert o.precision == B.FMG_FP64 and o.mode == B.FMG_PAPER


def test_workspace_bytes_plan():
    b2 = [B.workspace_bytes(2, 4, L) for L in range(1, 10)]
    assert all(x > 0 for x in b2) and all(a < b for a, b in zip(b2, b2[1:]))
    # three float64 arrays per level over the padded grids, plus small tables
    for L in (5, 9):
        nodes = sum((4 * 2 ** (k - 1) + 1) * (((4 * 2 ** (k - 1) + 1) + 15) // 16 * 16)
                    for k in range(1, L + 2))
        # plus the dense coarse-cycle operators of the levels with <= 1024 unknowns
        tail = 8 * sum(((4 * 2 ** (k - 1) - 1) ** 2) ** 2 for k in range(2, L + 2)
                       if (4 * 2 ** (k - 1) - 1) ** 2 <= 1024)
        assert 24 * nodes + tail <= B.workspace_bytes(2, 4, L) <= 24 * nodes + tail + 4 * 2 ** 20
    mixed = B.default_options(2, precision=B.FMG_MIXED)
    assert B.workspace_bytes(2, 4, 9, mixed) > B.workspace_bytes(2, 4, 9)
    assert B.workspace_bytes(3, 4, 6) > 0


@pytest.mark.parametrize("mesh", [(1, 4, 3), (4, 4, 3), (2, 1, 3), (2, 9, 3), (3, 5, 2), (2, 4, 0),
                                  (2, 4, 13), (3, 4, 9)])
def test_unsupported_meshes(mesh):
    assert B.workspace_bytes(*mesh) == 0
    h = ctypes.c_void_p()
    m = B.MeshDesc(*mesh)
    o = B.default_options(2)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: rejected before any device work
    rc = B.LIB.fmg_create_hierarchy(ctypes.byref(m), ctypes.byref(o), fake, 1 << 40, None, ctypes.byref(h))
    assert rc == B.FMG_E_UNSUPPORTED


@pytest.mark.parametrize("field,value", [("m_vcycles", 0), ("p_steps", 0), ("nu_pre", -1), ("smoother", 5),
                                         ("newton_max", 0), ("newton_tol", 0.0), ("precision", 3),
                                         ("mode", 7), ("cheb_lo", -1.0), ("newton_passes", 0)])
def test_invalid_options(field, value):
    o = B.default_options(2, **{field: value})
    assert B.workspace_bytes(2, 4, 3, o) == 0
    h = ctypes.c_void_p()
    m = B.MeshDesc(2, 4, 3)
    rc = B.LIB.fmg_create_hierarchy(ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(1 << 20), 1 << 40,
                                    None, ctypes.byref(h))
    assert rc == B.FMG_E_INVALID


def test_workspace_too_small_or_misaligned():
    m = B.MeshDesc(2, 4, 3)
    o = B.default_options(2)
    need = B.workspace_bytes(2, 4, 3)
    h = ctypes.c_void_p()
    rc = B.LIB.fmg_create_hierarchy(ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(1 << 20), need - 1,
                                    None, ctypes.byref(h))
    assert rc == B.FMG_E_WORKSPACE
    rc = B.LIB.fmg_create_hierarchy(ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p((1 << 20) + 8), need,
                                    None, ctypes.byref(h))
    assert rc == B.FMG_E_WORKSPACE


def test_null_arguments():
    h = ctypes.c_void_p()
    o = B.default_options(2)
    assert B.LIB.fmg_create_hierarchy(None, ctypes.byref(o), ctypes.c_void_p(1 << 20), 1 << 30, None,
                                      ctypes.byref(h)) == B.FMG_E_INVALID
    assert B.LIB.fmg_solve(None, None, None, None, None) == B.FMG_E_INVALID
    assert B.LIB.fmg_destroy(None) == B.FMG_E_INVALID
    assert B.LIB.fmg_get_report(None, None, None) == B.FMG_E_INVALID
    assert B.LIB.fmg_level_op(None, 0, 1, 0, None, None, None, 0.0, None) == B.FMG_E_INVALID
    assert B.LIB.fmg_solve_batch(None, None, None, None, -1, None) == B.FMG_E_INVALID
    assert B.LIB.fmg_solve_batch(None, None, None, None, 0, None) == B.FMG_OK


def test_status_strings():
    for code in range(7):
        assert B.status_str(code)
    assert B.status_str(99) == "unknown status"


def test_library_binds_to_torchs_hip_runtime():
    """Importing the binding maps exactly one HIP runtime (torch's): a second
    runtime would make torch's device pointers and streams foreign to the
    library."""
    maps = open("/proc/self/maps").read()
    runtimes = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(runtimes) == 1, runtimes


def test_noalloc_rejects_before_enqueueing():
    """fmg_solve_noalloc validates on the host and returns before any HIP call:
    invalid arguments, unsupported modes and problems larger than the static
    scratch (FMG_NOALLOC_SCRATCH_BYTES) are refused synchronously."""
    mesh = B.MeshDesc(2, 4, 9)                       # 2048^2: needs about 130 MiB
    fake = ctypes.c_void_p(0x1000)                   # never dereferenced
    prob = B.ProblemC(2, 0.0, fake)
    o = B.default_options(2)
    call = B.LIB.fmg_solve_noalloc
    assert call(ctypes.byref(mesh), ctypes.byref(o), ctypes.byref(prob), fake, None, None) == B.FMG_E_SCRATCH
    small = B.MeshDesc(2, 4, 3)
    assert call(None, ctypes.byref(o), ctypes.byref(prob), fake, None, None) == B.FMG_E_INVALID
    assert call(ctypes.byref(small), ctypes.byref(o), ctypes.byref(prob), None, None, None) == B.FMG_E_INVALID
    conv = B.default_options(2, mode=B.FMG_CONVERGED)
    assert call(ctypes.byref(small), ctypes.byref(conv), ctypes.byref(prob), fake, None, None) == \
        B.FMG_E_UNSUPPORTED
    fused = B.default_options(2, fuse_small_levels=1)
    assert call(ctypes.byref(small), ctypes.byref(fused), ctypes.byref(prob), fake, None, None) == \
        B.FMG_E_UNSUPPORTED
    elem = B.default_options(2, quadrature=B.FMG_QUAD_ELEMENT)
    assert call(ctypes.byref(small), ctypes.byref(elem), ctypes.byref(prob), fake, None, None) == \
        B.FMG_E_UNSUPPORTED
    bad = B.ProblemC(99, 0.0, fake)
    assert call(ctypes.byref(small), ctypes.byref(o), ctypes.byref(bad), fake, None, None) == B.FMG_E_INVALID
    assert B.status_str(B.FMG_E_SCRATCH).startswith("problem larger than the static scratch")


def test_element_rule_option_is_validated_on_the_host():
    """fmg_options.quadrature: vertex (default) or element; the element rule
    with the fused small-level kernel (vertex rule only) is refused."""
    assert B.default_options(2).quadrature == B.FMG_QUAD_VERTEX
    assert B.workspace_bytes(2, 4, 3, B.default_options(2, quadrature=B.FMG_QUAD_ELEMENT)) > 0
    assert B.workspace_bytes(3, 4, 2, B.default_options(3, quadrature=B.FMG_QUAD_ELEMENT)) > 0
    assert B.workspace_bytes(2, 4, 3, B.default_options(2, quadrature=2)) == 0
    assert B.workspace_bytes(2, 4, 3, B.default_options(2, quadrature=B.FMG_QUAD_ELEMENT,
                                                         fuse_small_levels=1)) == 0


def test_variable_coefficient_option_is_validated_on_the_host():
    """fmg_options.coefficients: identity (default) or variable; the variable
    operator needs float64, the vertex rule and no fused small levels; its
    workspace holds the stencil arrays of every level; fmg_set_coefficients
    and fmg_solve_noalloc refuse before any HIP call."""
    o = B.default_options(3)
    assert o.coefficients == B.FMG_COEF_IDENTITY
    var = B.default_options(3, coefficients=B.FMG_COEF_VARIABLE)
    base, big = B.workspace_bytes(3, 4, 4, o), B.workspace_bytes(3, 4, 4, var)
    nodes = 65 ** 3
    assert big - base >= 8 * 7 * nodes                   # seven forward-edge planes on the finest level
    assert B.workspace_bytes(2, 4, 3, B.default_options(2, coefficients=2)) == 0
    for bad in (dict(precision=B.FMG_MIXED), dict(quadrature=B.FMG_QUAD_ELEMENT), dict(fuse_small_levels=1)):
        assert B.workspace_bytes(2, 4, 3, B.default_options(2, coefficients=B.FMG_COEF_VARIABLE, **bad)) == 0
    fake = ctypes.c_void_p(0x1000)                       # never dereferenced
    assert B.LIB.fmg_set_coefficients(None, fake, None) == B.FMG_E_INVALID
    small = B.MeshDesc(2, 4, 3)
    prob = B.ProblemC(2, 0.0, fake)
    v2 = B.default_options(2, coefficients=B.FMG_COEF_VARIABLE)
    assert B.LIB.fmg_solve_noalloc(ctypes.byref(small), ctypes.byref(v2), ctypes.byref(prob), fake, None,
                                   None) == B.FMG_E_UNSUPPORTED
    weighted = B.ProblemC(2, 0.0, fake, fake)
    o2 = B.default_options(2)
    assert B.LIB.fmg_solve_noalloc(ctypes.byref(small), ctypes.byref(o2), ctypes.byref(weighted), fake, None,
                                   None) == B.FMG_E_UNSUPPORTED
