"""ctypes binding of the C ABI in include/fmg.h.

Argument marshalling only: every step of the solve runs in libfmg.so's HIP
kernels.  torch supplies device memory (the workspace, load and solution
tensors) and the stream.  Importing this module fails loudly if the library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
# torch is imported before the library is loaded: torch ships its own HIP
# runtime, and the library must bind to that same runtime (already mapped
# under the same soname).  Loaded the other way round, the process would hold
# two HIP runtimes and torch's device pointers and streams would be foreign
# to the library's.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FMG_LIBRARY", os.path.join(HERE, "libfmg.so"))

FMG_MAX_LEVELS = 16
FMG_OK, FMG_E_INVALID, FMG_E_UNSUPPORTED, FMG_E_WORKSPACE, FMG_E_HIP, FMG_E_NOT_CONVERGED, \
    FMG_E_NONFINITE, FMG_E_SCRATCH = range(8)
FMG_NOALLOC_SCRATCH_BYTES = 64 << 20
FMG_FP64, FMG_MIXED = 0, 1
FMG_SMOOTHER_DEFAULT, FMG_JACOBI, FMG_CHEBYSHEV = 0, 1, 2
FMG_PAPER, FMG_CONVERGED = 0, 1
FMG_QUAD_VERTEX, FMG_QUAD_ELEMENT = 0, 1
FMG_COEF_IDENTITY, FMG_COEF_VARIABLE = 0, 1
FMG_OP_APPLY_A, FMG_OP_SMOOTH, FMG_OP_RESTRICT, FMG_OP_PROLONG, FMG_OP_COARSE = range(5)

EXPORTED = ("fmg_default_options", "fmg_workspace_bytes", "fmg_create_hierarchy", "fmg_solve",
            "fmg_get_report", "fmg_solve_batch", "fmg_destroy", "fmg_status_str", "fmg_level_op",
            "fmg_profile_solve", "fmg_kernel_name", "fmg_time_level_kernel", "fmg_solve_noalloc",
            "fmg_set_coefficients")


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("coarse_cells", ctypes.c_int), ("refinements", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("m_vcycles", ctypes.c_int), ("p_steps", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("smoother", ctypes.c_int),
                ("omega", ctypes.c_double), ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("newton_max", ctypes.c_int), ("newton_tol", ctypes.c_double),
                ("newton_passes", ctypes.c_int), ("mode", ctypes.c_int),
                ("converged_max_steps", ctypes.c_int), ("converged_tol", ctypes.c_double),
                ("use_graph", ctypes.c_int), ("tail_max_nodes", ctypes.c_int),
                ("fuse_small_levels", ctypes.c_int), ("aug_max_blocks", ctypes.c_int),
                ("aug_small_nodes", ctypes.c_int), ("sweep_rows", ctypes.c_int),
                ("quadrature", ctypes.c_int), ("coefficients", ctypes.c_int)]


class ProblemC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("param", ctypes.c_double), ("g_nodes", ctypes.c_void_p),
                ("f_weight", ctypes.c_void_p)]


def _problem(kind, param, g, c=None) -> ProblemC:
    return ProblemC(int(kind), float(param), ctypes.c_void_p(g.data_ptr()),
                    ctypes.c_void_p(c.data_ptr() if c is not None else 0))


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("levels", ctypes.c_int), ("level1_iters", ctypes.c_int),
                ("extra_steps", ctypes.c_int),
                ("newton_iters", ctypes.c_int * FMG_MAX_LEVELS),
                ("newton_total", ctypes.c_int * FMG_MAX_LEVELS),
                ("alpha", ctypes.c_double * FMG_MAX_LEVELS),
                ("last_update_rel", ctypes.c_double)]

    def as_dict(self) -> dict:
        n = self.levels
        return {"status": self.status, "status_str": status_str(self.status), "levels": n,
                "level1_iters": self.level1_iters, "extra_steps": self.extra_steps,
                "newton_iters": list(self.newton_iters[:n]), "newton_total": list(self.newton_total[:n]),
                "alpha": list(self.alpha[:n]), "last_update_rel": self.last_update_rel}


FMG_PROFILE_MAX = 512


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("level", ctypes.c_int), ("launches", ctypes.c_int),
                ("nodes", ctypes.c_int), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("entries", ProfileEntry * FMG_PROFILE_MAX)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1611_05677_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.fmg_default_options.argtypes = [ctypes.c_int, P(Options)]
    lib.fmg_default_options.restype = None
    lib.fmg_workspace_bytes.argtypes = [P(MeshDesc), P(Options)]
    lib.fmg_workspace_bytes.restype = ctypes.c_size_t
    lib.fmg_create_hierarchy.argtypes = [P(MeshDesc), P(Options), vp, ctypes.c_size_t, vp, P(vp)]
    lib.fmg_create_hierarchy.restype = ctypes.c_int
    lib.fmg_solve.argtypes = [vp, P(ProblemC), vp, vp, vp]
    lib.fmg_solve.restype = ctypes.c_int
    lib.fmg_get_report.argtypes = [vp, P(Report), vp]
    lib.fmg_get_report.restype = ctypes.c_int
    lib.fmg_solve_batch.argtypes = [P(vp), P(ProblemC), P(vp), P(vp), ctypes.c_int, vp]
    lib.fmg_solve_batch.restype = ctypes.c_int
    lib.fmg_destroy.argtypes = [vp]
    lib.fmg_destroy.restype = ctypes.c_int
    lib.fmg_status_str.argtypes = [ctypes.c_int]
    lib.fmg_status_str.restype = ctypes.c_char_p
    lib.fmg_level_op.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp]
    lib.fmg_level_op.restype = ctypes.c_int
    lib.fmg_profile_solve.argtypes = [vp, P(ProblemC), vp, vp, P(Profile)]
    lib.fmg_profile_solve.restype = ctypes.c_int
    lib.fmg_kernel_name.argtypes = [ctypes.c_int]
    lib.fmg_kernel_name.restype = ctypes.c_char_p
    lib.fmg_time_level_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                          P(ctypes.c_double), P(ctypes.c_double)]
    lib.fmg_time_level_kernel.restype = ctypes.c_int
    lib.fmg_solve_noalloc.argtypes = [P(MeshDesc), P(Options), P(ProblemC), vp, vp, vp]
    lib.fmg_solve_noalloc.restype = ctypes.c_int
    lib.fmg_set_coefficients.argtypes = [vp, vp, vp]
    lib.fmg_set_coefficients.restype = ctypes.c_int
    return lib


LIB = _load()


class FMGError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_str(code)} ({code})")
        self.code = code


def kernel_name(kernel: int) -> str:
    return LIB.fmg_kernel_name(int(kernel)).decode()


def status_str(code: int) -> str:
    return LIB.fmg_status_str(int(code)).decode()


def _check(code: int, where: str):
    if code != FMG_OK:
        raise FMGError(code, where)


def default_options(dim: int, **overrides) -> Options:
    o = Options()
    LIB.fmg_default_options(int(dim), ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def workspace_bytes(dim: int, coarse_cells: int, refinements: int, opts: Options | None = None) -> int:
    mesh = MeshDesc(dim, coarse_cells, refinements)
    o = opts if opts is not None else default_options(dim)
    return int(LIB.fmg_workspace_bytes(ctypes.byref(mesh), ctypes.byref(o)))


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Hierarchy:
    """A planned level hierarchy living in a caller-owned device workspace."""

    def __init__(self, dim: int, coarse_cells: int, refinements: int, opts: Options | None = None,
                 workspace=None, device: str = "cuda", stream=None):
        import torch
        self.dim, self.coarse_cells, self.refinements = dim, coarse_cells, refinements
        self.opts = opts if opts is not None else default_options(dim)
        self.mesh = MeshDesc(dim, coarse_cells, refinements)
        self.nbytes = int(LIB.fmg_workspace_bytes(ctypes.byref(self.mesh), ctypes.byref(self.opts)))
        if self.nbytes == 0:
            raise FMGError(FMG_E_UNSUPPORTED, "fmg_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.workspace = workspace
        self.stream = stream
        h = ctypes.c_void_p()
        _check(LIB.fmg_create_hierarchy(ctypes.byref(self.mesh), ctypes.byref(self.opts),
                                        ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(self.nbytes),
                                        ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)),
               "fmg_create_hierarchy")
        self.handle = h

    @property
    def n(self) -> int:
        return self.coarse_cells * 2 ** self.refinements

    @property
    def levels(self) -> int:
        return self.refinements + 1

    def nodes(self, level: int | None = None) -> int:
        k = self.levels if level is None else level
        return (self.coarse_cells * 2 ** (k - 1) + 1) ** self.dim

    def set_coefficients(self, coef, stream=None):
        """FMG_COEF_VARIABLE hierarchies: the matrix A(x) per finest cell as a
        contiguous float64 device tensor of d(d+1)/2 component planes of n^d
        cells (upper triangle row by row).  Stream-ordered; `coef` must stay
        alive until the setup kernels have run (the call keeps a reference)."""
        import torch
        ncomp = self.dim * (self.dim + 1) // 2
        if coef.dtype != torch.float64 or not coef.is_contiguous() or coef.numel() != ncomp * self.n ** self.dim:
            raise ValueError("coef must be a contiguous float64 tensor of d(d+1)/2 planes of n^d cells")
        st = stream if stream is not None else self.stream
        _check(LIB.fmg_set_coefficients(self.handle, ctypes.c_void_p(coef.data_ptr()),
                                        ctypes.c_void_p(_stream_ptr(st))), "fmg_set_coefficients")
        self._coef = coef

    def solve_async(self, g, kind: int, param: float = 0.0, out=None, report_ptr: int = 0, stream=None,
                    c=None):
        """Enqueue one solve on `stream` (default: the hierarchy's stream, else
        torch's current one); returns the output tensor.  c: optional weight
        c(x) of f(x, u) = c(x) f(u) at the finest nodes (variable-coefficient
        hierarchies)."""
        import torch
        if out is None:
            out = torch.empty(self.nodes(), dtype=torch.float64, device=g.device)
        if g.dtype != torch.float64 or not g.is_contiguous() or g.numel() != self.nodes():
            raise ValueError("g must be a contiguous float64 tensor with (n+1)^d entries")
        if c is not None and (c.dtype != torch.float64 or not c.is_contiguous() or c.numel() != self.nodes()):
            raise ValueError("c must be a contiguous float64 tensor with (n+1)^d entries")
        prob = _problem(kind, param, g, c)
        st = stream if stream is not None else self.stream
        _check(LIB.fmg_solve(self.handle, ctypes.byref(prob), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(report_ptr), ctypes.c_void_p(_stream_ptr(st))),
               "fmg_solve")
        return out

    def report(self, stream=None) -> dict:
        """Report of the last solve (synchronises `stream`)."""
        r = Report()
        st = stream if stream is not None else self.stream
        _check(LIB.fmg_get_report(self.handle, ctypes.byref(r), ctypes.c_void_p(_stream_ptr(st))),
               "fmg_get_report")
        return r.as_dict()

    def solve(self, g, kind: int, param: float = 0.0, out=None, c=None):
        out = self.solve_async(g, kind, param, out, c=c)
        return out, self.report()

    def level_op(self, op: int, level: int, in0, in1=None, precision: int = FMG_FP64, omega: float = 0.0):
        import torch
        lev_nodes = self.nodes(level - 1 if op == FMG_OP_RESTRICT else level)
        out = torch.empty(lev_nodes, dtype=torch.float64, device=in0.device)
        _check(LIB.fmg_level_op(self.handle, int(op), int(level), int(precision),
                                ctypes.c_void_p(in0.data_ptr()),
                                ctypes.c_void_p(in1.data_ptr() if in1 is not None else 0),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_double(omega),
                                ctypes.c_void_p(_stream_ptr(self.stream))), "fmg_level_op")
        return out

    def close(self):
        if getattr(self, "handle", None):
            LIB.fmg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(hs: list, gs: list, kinds: list, params: list, outs: list, stream=None):
    """Enqueue several independent solves (distinct hierarchies and outputs) as
    one graph launch on `stream`; the solves run side by side on the device."""
    n = len(hs)
    H = (ctypes.c_void_p * n)(*[h.handle for h in hs])
    P = (ProblemC * n)(*[_problem(k, p, g) for g, k, p in zip(gs, kinds, params)])
    O = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(LIB.fmg_solve_batch(H, P, O, None, n, ctypes.c_void_p(_stream_ptr(stream))), "fmg_solve_batch")


def solve_noalloc(dim: int, coarse_cells: int, refinements: int, g, kind: int, param: float = 0.0,
                  opts: Options | None = None, out=None, report=None, stream=None):
    """One solve through fmg_solve_noalloc (the library's static scratch as
    workspace; no device allocation inside the call).  `out` (float64,
    (n+1)^d) and `report` (a device uint8 tensor of sizeof(fmg_report) bytes)
    are caller-owned and may be preallocated; returns `out`."""
    import torch
    nodes = (coarse_cells * 2 ** refinements + 1) ** dim
    if out is None:
        out = torch.empty(nodes, dtype=torch.float64, device=g.device)
    if g.dtype != torch.float64 or not g.is_contiguous() or g.numel() != nodes:
        raise ValueError("g must be a contiguous float64 tensor with (n+1)^d entries")
    mesh = MeshDesc(dim, coarse_cells, refinements)
    o = opts if opts is not None else default_options(dim)
    prob = _problem(kind, param, g)
    _check(LIB.fmg_solve_noalloc(ctypes.byref(mesh), ctypes.byref(o), ctypes.byref(prob),
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(report.data_ptr() if report is not None else 0),
                                 ctypes.c_void_p(_stream_ptr(stream))), "fmg_solve_noalloc")
    return out


def report_from_device(buf) -> dict:
    """Decode an fmg_report written by the device into a uint8 tensor."""
    raw = bytes(buf.cpu().numpy().tobytes())
    r = Report.from_buffer_copy(raw[:ctypes.sizeof(Report)])
    return r.as_dict()


def kernel_id(name: str) -> int:
    """Kernel class id of a kernel name reported by fmg_kernel_name."""
    for k in range(256):
        nm = kernel_name(k)
        if nm == name:
            return k
        if nm == "unknown":
            break
    raise KeyError(name)


def time_level_kernel(h: "Hierarchy", name: str, level: int, reps: int, stream=None) -> tuple[float, float]:
    """(ms per launch, algorithmic bytes per launch) of one level kernel."""
    ms, nb = ctypes.c_double(), ctypes.c_double()
    _check(LIB.fmg_time_level_kernel(h.handle, kernel_id(name), int(level), int(reps),
                                     ctypes.c_void_p(_stream_ptr(stream if stream is not None else h.stream)),
                                     ctypes.byref(ms), ctypes.byref(nb)), "fmg_time_level_kernel")
    return ms.value, nb.value


def exported_symbols() -> list[str]:
    return [s for s in EXPORTED if hasattr(LIB, s)]
