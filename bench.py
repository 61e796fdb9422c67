"""Throughput of the full-multigrid semilinear solver on one MI355X.

Workload: 2D unit square, P1 on right triangles, coarse 4x4 grid refined 9
times (2048x2048 cells, 4,190,209 interior DOFs); -Laplace(u) + u^3 = g with g
manufactured from u = sin(pi x) sin(pi y) exp(x); Algorithm 3.2 with m = 2
V(2,2)-cycles and p = 1 correction step per level.  One step = one complete
solve (all levels, V-cycles, augmented-space Newton solves), inputs resident
in HBM.  Reported: fine DOF/s of the plain float64 path (`value`) and of the
mixed path (float32 cycles inside float64 refinement), per-solve latency
p50/p99 from HIP events, the accuracy gate against the stored oracle values,
the roofline of the dominant kernel from live HIP-event timing, and the CPU
oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine DOF/s solved to discretization error, plain vs mixed; p50/p99 latency"
GOLDEN = os.path.join(ROOT, "tests", "golden", "fmg_reference.json")
HBM_PEAK_GBS = 8000.0
# name -> (description, problem factory, golden key, disc scale from the golden level)
WORKLOADS = {
    "square2048": ("2D unit square, P1 right triangles, coarse 4x4 refined 9 times (2048x2048, "
                   "4,190,209 DOFs); -Lap u + u^3 = g, g manufactured from u = sin(pi x) sin(pi y) exp(x); "
                   "m = 2 V(2,2) cycles, p = 1", "square_cubic_sin_expx", 9, "square_cubic_sin_expx_L9", 1.0),
    "cube256": ("3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 6 times (256^3, 16,581,375 DOFs); "
                "-Lap u + u + sin u = g, g manufactured from u = sin(pi x) sin(pi y) sin(pi z); "
                "m = 2 V(2,2) Chebyshev-weighted cycles, p = 1", "cube_u_plus_sin", 6, "cube_u_plus_sin_L5", 0.25),
    "cube128": ("3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 5 times (128^3, 2,048,383 DOFs); "
                "-Lap u + u + sin u = g, g manufactured from u = sin(pi x) sin(pi y) sin(pi z)",
                "cube_u_plus_sin", 5, "cube_u_plus_sin_L5", 1.0),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q))


def run_mode(B, torch, P, g, precision, steps, warmup, golden, disc_scale=1.0):
    opts = B.default_options(P.dim, precision=precision)
    H = B.Hierarchy(P.dim, P.coarse_cells, P.refinements, opts, device="cuda:0")
    out = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        H.solve_async(g, P.f_kind, P.f_param, out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        H.solve_async(g, P.f_kind, P.f_param, out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in ev]
    rep = H.report()
    u = out.cpu().numpy()
    # accuracy gate against the stored oracle values (at the golden level; for a
    # deeper level the discretisation error is extrapolated by the O(h^2) rate)
    shape = (P.n + 1,) * P.dim
    inner = tuple(slice(1, -1) for _ in range(P.dim))
    interior = P.u_exact_nodes.reshape(shape)[inner].ravel()
    uint = u.reshape(shape)[inner].ravel()
    exact_err = float(np.sqrt(np.sum((uint - interior) ** 2) / P.n ** P.dim))
    disc = golden["disc_nodal_l2"] * disc_scale
    same_level = golden["n"] == P.n
    idx = np.asarray(golden["sample_idx"]) if same_level else np.zeros(0, dtype=np.int64)
    conv = np.asarray(golden["converged_sample"]) if same_level else np.zeros(0)
    paper = np.asarray(golden["paper_sample"]) if same_level else np.zeros(0)
    scale = np.max(np.abs(conv)) if same_level else 1.0
    res = {
        "dof_per_s": P.interior_dofs / (wall / steps),
        "ms_per_solve": 1e3 * wall / steps,
        "latency_ms_p50": percentile(lat, 50), "latency_ms_p99": percentile(lat, 99),
        "status": rep["status"], "newton_iters": rep["newton_iters"],
        "err_vs_exact_nodal_l2": exact_err, "disc_nodal_l2": disc,
        "gate_total_le_1.1disc": bool(exact_err <= 1.1 * disc),
        "disc_source": "oracle" if same_level else "oracle one level coarser / 4 (O(h^2))",
    }
    if same_level:
        res["sample_maxrel_vs_oracle_paper"] = float(np.max(np.abs(u[idx] - paper)) / scale)
        res["sample_maxrel_vs_oracle_converged"] = float(np.max(np.abs(u[idx] - conv)) / scale)
        res["norm2_rel_vs_oracle_paper"] = abs(float(np.linalg.norm(u)) - golden["paper_norm2"]) / golden["paper_norm2"]
        # algebraic error estimate at the sample nodes, relative to disc
        res["alg_over_disc_sampled"] = float(np.sqrt(np.mean((u[idx] - conv) ** 2)) /
                                             max(np.sqrt(np.mean((conv - P.u_exact_nodes[idx]) ** 2)), 1e-300))
    res["gate_pass"] = bool(res["gate_total_le_1.1disc"] and rep["status"] == 0 and
                            res.get("alg_over_disc_sampled", 0.0) <= 0.5)
    return H, res


def profile_mode(B, H, P, g, torch):
    """Per-kernel HIP-event timing of one direct-launch solve (same stream)."""
    import ctypes
    prof = B.Profile()
    out = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
    prob = B.ProblemC(int(P.f_kind), float(P.f_param), ctypes.c_void_p(g.data_ptr()))
    B._check(B.LIB.fmg_profile_solve(H.handle, ctypes.byref(prob), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     ctypes.byref(prof)), "fmg_profile_solve")
    rows = []
    for e in prof.entries[:prof.count]:
        rows.append({"kernel": B.kernel_name(e.kernel), "level": e.level, "launches": e.launches,
                     "nodes": e.nodes, "ms": e.ms, "bytes": e.bytes})
    return prof.total_ms, rows


def roofline_from_profile(rows, finest):
    """Dominant bandwidth kernel (most event time among the kernels that stream
    nodal arrays) and its launches on the finest level."""
    by_kernel, streaming = {}, {}
    for r in rows:
        by_kernel[r["kernel"]] = by_kernel.get(r["kernel"], 0.0) + r["ms"]
        if r["bytes"] > 0:
            streaming[r["kernel"]] = streaming.get(r["kernel"], 0.0) + r["ms"]
    total = sum(by_kernel.values())
    dominant = max(streaming, key=streaming.get)
    fine = [r for r in rows if r["kernel"] == dominant and r["level"] == finest]
    if not fine or fine[0]["bytes"] <= 0:
        return None, by_kernel, total
    f = fine[0]
    avg_s = f["ms"] / f["launches"] / 1e3
    bytes_per_launch = f["bytes"] / f["launches"]
    achieved = bytes_per_launch / avg_s / 1e9
    roof = {"bound": "hbm", "kernel": dominant, "level": finest, "launches_timed": f["launches"],
            "avg_launch_us": avg_s * 1e6, "bytes_per_launch": bytes_per_launch,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None, "share_of_solve_time": by_kernel[dominant] / total}
    return roof, by_kernel, total


def cpu_baseline(P, W):
    """The CPU oracle (replica of the FMG scheme) on the same workload: the solve
    is timed, the hierarchy build (analogue of fmg_create_hierarchy) is not.
    3D runs one level coarser (the oracle's assembly does not fit otherwise)."""
    from oracle.nonlinear import Nonlinearity
    from oracle.o2 import Hierarchy as O2H
    from oracle.o2 import fmg as o2_fmg
    full = P
    if P.dim == 3 and P.refinements > 4:
        P = W.cube_u_plus_sin(4)
    t0 = time.perf_counter()
    H = O2H(P.dim, P.coarse_cells, P.refinements)
    build_s = time.perf_counter() - t0
    nl = Nonlinearity(P.f_kind, P.f_param)
    t0 = time.perf_counter()
    o2_fmg(H, P.g_nodes, nl)
    solve_s = time.perf_counter() - t0
    return {"value": P.interior_dofs / solve_s, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of {P.name} ({P.interior_dofs} DOFs"
                      f"{'' if P is full else ', a coarser instance of the benchmark problem'}) by the "
                      f"oracle's CPU replica of the FMG scheme (scipy CSR, single thread); solve {solve_s:.2f} s, "
                      f"hierarchy assembly {build_s:.1f} s not timed",
            "host_cpu_count": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", default="square2048", choices=sorted(WORKLOADS))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver runs on a single "
              "device and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    from paper_1611_05677_amd import build as build_mod
    if not os.path.exists(build_mod.LIB):
        build_mod.build()
    import torch

    from paper_1611_05677_amd import binding as B
    from paper_1611_05677_amd import workloads as W

    desc, factory, depth, gkey, disc_scale = WORKLOADS[args.workload]
    golden = json.load(open(GOLDEN))[gkey]
    P = getattr(W, factory)(depth)
    g = torch.from_numpy(P.g_nodes).to("cuda:0")
    log(f"workload: {P.name} n={P.n} DOFs={P.interior_dofs}")
    modes = {}
    hier = {}
    for name, prec in (("fp64", B.FMG_FP64), ("mixed", B.FMG_MIXED)):
        H, res = run_mode(B, torch, P, g, prec, args.steps, args.warmup, golden, disc_scale)
        modes[name] = res
        hier[name] = H
        log(f"{name}: {res['ms_per_solve']:.3f} ms/solve, {res['dof_per_s'] / 1e9:.3f} GDOF/s, "
            f"p50 {res['latency_ms_p50']:.3f} ms p99 {res['latency_ms_p99']:.3f} ms, gate {res['gate_pass']}")
    roof = None
    if not args.no_profile:
        for name in ("fp64", "mixed"):
            total_ms, rows = profile_mode(B, hier[name], P, g, torch)
            r, by_kernel, tot = roofline_from_profile(rows, P.n_levels)
            modes[name]["profile_event_ms_total"] = total_ms
            modes[name]["profile_rows"] = sorted(rows, key=lambda r: -r["ms"])[:40]
            modes[name]["profile_ms_by_kernel"] = {k: round(v, 4) for k, v in
                                                   sorted(by_kernel.items(), key=lambda kv: -kv[1])}
            if name == "fp64":
                roof = r
            modes[name]["roofline_dominant"] = r
    primary = modes["fp64"]
    line = {
        "metric": METRIC, "value": primary["dof_per_s"], "unit": "DOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": primary["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "dofs": P.interior_dofs, "levels": P.n_levels,
                   "precision_of_value": "fp64 (plain)"},
        "latency_ms_p50": primary["latency_ms_p50"], "latency_ms_p99": primary["latency_ms_p99"],
        "mixed": {k: modes["mixed"][k] for k in ("dof_per_s", "ms_per_solve", "latency_ms_p50",
                                                 "latency_ms_p99", "gate_pass")},
        "mixed_speedup_vs_fp64": modes["mixed"]["dof_per_s"] / primary["dof_per_s"],
        "modes": modes,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        line["cpu_baseline"] = cpu_baseline(P, W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
