"""Throughput of the full-multigrid semilinear solver on one MI355X.

Default workload (the largest single-GPU configuration): 3D unit cube, Kuhn
tetrahedra, coarse 4^3 grid refined 6 times (256^3 cells, 16,581,375 interior
DOFs); -Laplace(u) + u + sin(u) = g with g manufactured from
u = sin(pi x) sin(pi y) sin(pi z); Algorithm 3.2 with m = 2 V(2,2) cycles
(Chebyshev-weighted Jacobi) and p = 1 correction step per level.  One step =
one complete solve (all levels, V-cycles, augmented-space Newton solves),
inputs resident in HBM.  Reported: fine DOF/s of the plain float64 path
(`value`) and of the mixed path (float32 cycles inside float64 refinement),
per-solve latency p50/p99 from HIP events, the accuracy gate (both conditions,
every node) against the stored oracle values at the same level, the HBM
roofline of the dominant streaming kernel and the float64 ALU roofline of the
fine quadrature pass (live HIP-event timing, counter-derived bytes and
flops), the 2D 2048^2 configuration as a secondary record, and the CPU oracle
timed on the host.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--workload NAME]
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
FP64_VALU_PEAK_TFLOPS = 78.6
# name -> (description, problem factory, refinements, golden key at the same level)
WORKLOADS = {
    "cube256": ("3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 6 times (256^3, 16,581,375 DOFs); "
                "-Lap u + u + sin u = g, g manufactured from u = sin(pi x) sin(pi y) sin(pi z); "
                "m = 2 V(2,2) Chebyshev-weighted cycles, p = 1", "cube_u_plus_sin", 6, "cube_u_plus_sin_L6"),
    "square2048": ("2D unit square, P1 right triangles, coarse 4x4 refined 9 times (2048x2048, "
                   "4,190,209 DOFs); -Lap u + u^3 = g, g manufactured from u = sin(pi x) sin(pi y) exp(x); "
                   "m = 2 V(2,2) cycles, p = 1", "square_cubic_sin_expx", 9, "square_cubic_sin_expx_L9"),
    "cube128": ("3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 5 times (128^3, 2,048,383 DOFs); "
                "-Lap u + u + sin u = g, g manufactured from u = sin(pi x) sin(pi y) sin(pi z)",
                "cube_u_plus_sin", 5, "cube_u_plus_sin_L5"),
}
SECONDARY = {"cube256": "square2048"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q))


def nodal(P, v):
    return float(np.sqrt((1.0 / P.n) ** P.dim * np.sum(v * v)))


def converged_solution(B, torch, P, g, golden):
    """ubar_h from the library's converged mode (float64), checked against the
    oracle's converged solution at the stored sample nodes."""
    H = B.Hierarchy(P.dim, P.coarse_cells, P.refinements, B.default_options(P.dim, mode=B.FMG_CONVERGED),
                    device="cuda:0")
    u, rep = H.solve(g, P.f_kind, P.f_param)
    H.close()
    uc = u.cpu().numpy()
    idx = np.asarray(golden["sample_idx"], dtype=np.int64)
    conv = np.asarray(golden["converged_sample"])
    info = {"status": rep["status"], "extra_steps": rep["extra_steps"],
            "last_update_rel": rep["last_update_rel"],
            "sample_maxrel_vs_oracle_converged": float(np.max(np.abs(uc[idx] - conv)) / np.max(np.abs(conv)))}
    return uc, info


def run_mode(B, torch, P, g, precision, steps, warmup, golden, uc):
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
    # accuracy gate over every node, against the oracle's discretisation error
    # at this level (ubar_h: the library's converged-mode solve, checked against
    # the oracle's converged solution)
    exact_err = nodal(P, u - P.u_exact_nodes)
    disc = golden["disc_nodal_l2"]
    alg = nodal(P, u - uc)
    idx = np.asarray(golden["sample_idx"], dtype=np.int64)
    paper = np.asarray(golden["paper_sample"])
    res = {
        "dof_per_s": P.interior_dofs / (wall / steps),
        "ms_per_solve": 1e3 * wall / steps,
        "latency_ms_p50": percentile(lat, 50), "latency_ms_p99": percentile(lat, 99),
        "status": rep["status"], "newton_iters": rep["newton_iters"],
        "err_vs_exact_nodal_l2": exact_err, "disc_nodal_l2": disc,
        "disc_source": "oracle, same level (ubar_h of the oracle's converged mode)",
        "alg_nodal_l2": alg, "alg_over_disc": alg / disc,
        "alg_nodal_l2_oracle_fp64": golden["alg_nodal_l2"],
        "gate_total_le_1.1disc": bool(exact_err <= 1.1 * disc),
        "gate_alg_le_0.5disc": bool(alg <= 0.5 * disc),
        "sample_maxrel_vs_oracle_paper": float(np.max(np.abs(u[idx] - paper)) / np.max(np.abs(paper))),
        "norm2_rel_vs_oracle_paper": abs(float(np.linalg.norm(u)) - golden["paper_norm2"]) / golden["paper_norm2"],
    }
    res["gate_pass"] = bool(res["gate_total_le_1.1disc"] and res["gate_alg_le_0.5disc"] and rep["status"] == 0)
    return H, res


def profile_mode(B, H, P, g, torch, c=None):
    """Per-kernel HIP-event timing of one direct-launch solve (same stream)."""
    import ctypes
    prof = B.Profile()
    out = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
    prob = B._problem(P.f_kind, P.f_param, g, c)
    B._check(B.LIB.fmg_profile_solve(H.handle, ctypes.byref(prob), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     ctypes.byref(prof)), "fmg_profile_solve")
    rows = []
    for e in prof.entries[:prof.count]:
        rows.append({"kernel": B.kernel_name(e.kernel), "level": e.level, "launches": e.launches,
                     "nodes": e.nodes, "ms": e.ms, "bytes": e.bytes})
    return prof.total_ms, rows


# dominant streaming kernel per dimension (the V-cycle level kernel that moves
# the most bytes) and the source file that defines it
ROOF_KERNEL = {2: ("pre_sweeps_restrict_2d_stream_f64", "fmg_kernels_stream2d.h"),
               3: ("pre_sweep_pair_3d_f64", "fmg_kernels_pair3d.h")}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
FLOPS_FILE = os.path.join(ROOT, "profiles", "pmc_flops.json")
# the fine quadrature pass of the augmented problem (float64 ALU bound)
ALU_KERNEL = ("aug_pass", "fmg_kernels_aug.h")


def kernel_source_hash(fname):
    import hashlib
    path = os.path.join(ROOT, "paper_1611_05677_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _counter_entry(path, kernel, workload, fname):
    """A committed rocprofv3 counter record for this kernel and workload, if it
    was taken on the current source of the kernel."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    for e in rec.get("entries", []):
        if e["kernel"] == kernel and e["workload"] == workload and e["source_sha256_16"] == kernel_source_hash(fname):
            return e
    return None


def roofline_live(B, H, dim, workload, reps, stream=None):
    """Mean launch duration of the dominant kernel at the finest level, timed
    with HIP events around `reps` back-to-back launches on the bench stream."""
    name, fname = ROOF_KERNEL[dim]
    ms, nbytes = B.time_level_kernel(H, name, H.levels, reps, stream)
    achieved = nbytes / (ms * 1e-3) / 1e9
    e = _counter_entry(TRAFFIC_FILE, name, workload, fname)
    traffic = e["hbm_bytes_per_launch"] if e else None
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": name, "level": H.levels,
           "launches_timed": reps, "avg_launch_us": ms * 1e3, "bytes_per_launch": nbytes,
           "bytes_model": "each nodal array of the launch read or written once: "
                          + ("s(3N + N_c), N, N_c interior nodes of the level and of the next coarser"
                             if dim == 2 else "3sN (read x, b; write x2 after two sweeps), N interior nodes "
                                              "of the level"),
           "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if traffic is not None else None}
    if dim == 2:
        # the 2048^2 working set (x, b, x', b_c: about 109 MB) stays in the 256 MB
        # Infinity Cache across back-to-back launches: not an HBM measurement
        out["bound"] = "effective"
        out["note"] = ("working set below the 256 MB Infinity Cache: effective GB/s of algorithmic bytes, "
                       "not a fraction of HBM bandwidth")
    return out


def alu_roofline(rows, workload, level, dim, kernel=ALU_KERNEL):
    """Float64 rate of the fine quadrature pass at the finest level: executed
    float64 FLOPs per launch from the committed counter run (VALU float64
    instructions x 64 lanes, FMA counted twice) over the mean launch duration
    from the event-bracketed profile of the same solve."""
    name, fname = kernel
    r = [x for x in rows if x["kernel"] == name and x["level"] == level]
    if not r or r[0]["launches"] == 0:
        return None
    avg_ms = r[0]["ms"] / r[0]["launches"]
    e = _counter_entry(FLOPS_FILE, name, workload, fname)
    flops = e["fp64_flop_per_launch"] if e else None
    out = {"bound": "alu", "kernel": name, "level": level, "avg_launch_us": avg_ms * 1e3,
           "launches": r[0]["launches"], "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "achieved": None, "frac": None, "traffic": None, "flop_per_launch": flops,
           "flop_source": os.path.relpath(FLOPS_FILE, ROOT) if e else None,
           "fine_nodes": r[0]["nodes"], "bytes_per_launch": r[0]["bytes"]}
    if flops:
        out["achieved"] = flops / (avg_ms * 1e-3) / 1e12
        out["frac"] = out["achieved"] / FP64_VALU_PEAK_TFLOPS
        out["flop_per_node"] = flops / max(1, r[0]["nodes"])
        out["counters"] = e.get("counters")
    out["achieved_gbs"] = r[0]["bytes"] / r[0]["launches"] / (avg_ms * 1e-3) / 1e9
    return out


def roofline_from_profile(rows):
    """Device time per kernel class from the event-bracketed profile (each
    launch inflated by the event pair: shares, not durations)."""
    by_kernel = {}
    for r in rows:
        by_kernel[r["kernel"]] = by_kernel.get(r["kernel"], 0.0) + r["ms"]
    return by_kernel


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(P, W):
    """The CPU oracle timed on the host, single thread (BLAS pools limited to
    one thread): O2, the oracle's replica of the FMG scheme (the same
    algorithm), and O1, the fine-space Newton solve of the discrete problem
    (the non-multigrid baseline), on a bounded sample of the benchmark's
    problem family: the same manufactured problem one or two levels coarser,
    so that the leg takes tens of seconds.  The hierarchy assembly (analogue of
    fmg_create_hierarchy) is not timed; O2 is the median of three solves."""
    from threadpoolctl import threadpool_limits

    from oracle.nonlinear import Nonlinearity
    from oracle.o1 import solve_fine
    from oracle.o2 import Hierarchy as O2H
    from oracle.o2 import fmg as o2_fmg
    factory = W.cube_u_plus_sin if P.dim == 3 else W.square_cubic_sin_expx
    S2 = factory(P.refinements - 1)          # O2: one level coarser
    S1 = factory(P.refinements - 2)          # O1: two levels coarser (its CG Newton costs more per DOF)
    with threadpool_limits(limits=1):
        nl = Nonlinearity(S2.f_kind, S2.f_param)
        t0 = time.perf_counter()
        H = O2H(S2.dim, S2.coarse_cells, S2.refinements)
        build_s = time.perf_counter() - t0
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            o2_fmg(H, S2.g_nodes, nl)
            times.append(time.perf_counter() - t0)
        o2_s = float(np.median(times))
        del H
        t0 = time.perf_counter()
        o1 = solve_fine(S1.dim, S1.n, S1.g_nodes, Nonlinearity(S1.f_kind, S1.f_param))
        o1_s = time.perf_counter() - t0
    return {"value": S2.interior_dofs / o2_s, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"O2 (the oracle's CPU replica of the FMG scheme, scipy CSR): {S2.name} "
                      f"({S2.interior_dofs} DOFs, the benchmark's manufactured problem one level coarser), "
                      f"median of 3 solves {o2_s:.3f} s, hierarchy assembly {build_s:.1f} s not timed; "
                      f"O1 (fine-space Newton, {o1.iterations} iterations): {S1.name} ({S1.interior_dofs} DOFs, "
                      f"two levels coarser) {o1_s:.2f} s",
            "o2_dof_per_s": S2.interior_dofs / o2_s, "o2_solve_s": o2_s, "o2_dofs": S2.interior_dofs,
            "o1_dof_per_s": S1.interior_dofs / o1_s, "o1_solve_s": o1_s, "o1_dofs": S1.interior_dofs,
            "o1_newton_iterations": o1.iterations,
            "cpu_model": _cpu_model(), "host_cpu_count": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "threads_env": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                            "MKL_NUM_THREADS")},
            "threads_used": "1 (scipy sparse kernels are single-threaded; BLAS pools limited to 1)"}


BATCH_DESC = ("batched: 64 independent 2D unit-square problems, depths U{6..10} (seeded), f = u^3, "
              "g = random Fourier series (16x16 modes, N(0,1)/(1+|k|^2)), mixed precision, one graph launch")
SERVE_DESC = ("serving: Poisson arrivals (seeded; 200 req/s unless --rate says otherwise) mixing 2D (depths 7-10) and 3D (coarse 4^3 refined "
              "3-6 times), f in {u^3, u+sin u, |u|u}, random-Fourier g, resident hierarchies, admission by "
              "device-memory footprint (64 GB), mixed precision")


def batch_mode(args, B, W, torch):
    """64 problems in one graph launch vs. the same solves one after another."""
    specs = W.batched_specs()
    prec = B.FMG_MIXED
    hs, gs, outs = [], [], []
    for d, seed in specs:
        h = B.Hierarchy(2, 4, d, B.default_options(2, precision=prec), device="cuda:0")
        hs.append(h)
        gs.append(W.fourier_load_device(W.fourier_coefficients(2, 16, seed), h.n, "cuda:0"))
        outs.append(torch.empty(h.nodes(), dtype=torch.float64, device="cuda:0"))
    dofs = sum((h.n - 1) ** 2 for h in hs)
    kinds, params = [W.F_CUBIC] * len(hs), [0.0] * len(hs)
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, [a.elapsed_time(b) for a, b in ev]

    def batched():
        B.solve_batch(hs, gs, kinds, params, outs)

    def sequential():
        for h, g, o in zip(hs, gs, outs):
            h.solve_async(g, W.F_CUBIC, 0.0, o)

    for _ in range(max(1, args.warmup)):
        batched()
        sequential()
    torch.cuda.synchronize()
    tb, lat_b = timed(batched, args.steps)
    statuses = [h.report()["status"] for h in hs]
    batch_res = [o.clone() for o in outs]
    ts, lat_s = timed(sequential, max(1, args.steps // 2))
    same = all(torch.equal(a, b) for a, b in zip(batch_res, outs))
    # accuracy: a few members against the float64 path solved alone
    diffs = []
    for i in sorted(range(len(hs)), key=lambda i: hs[i].n)[:4]:
        h64 = B.Hierarchy(2, 4, hs[i].refinements, B.default_options(2), device="cuda:0")
        u64, _ = h64.solve(gs[i], W.F_CUBIC)
        h64.close()
        diffs.append(float(torch.linalg.norm(batch_res[i] - u64) / torch.linalg.norm(u64)))
    for h in hs:
        h.close()
    depth_hist = {int(d): sum(1 for dd, _ in specs if dd == d) for d in sorted({d for d, _ in specs})}
    return {
        "metric": METRIC, "value": dofs / tb, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tb * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": BATCH_DESC, "problems": len(hs), "total_dofs": dofs, "depths": depth_hist},
        "latency_ms_p50": percentile(lat_b, 50), "latency_ms_p99": percentile(lat_b, 99),
        "sequential": {"dof_per_s": dofs / ts, "ms_per_batch": ts * 1e3},
        "batched_speedup_vs_sequential": ts / tb,
        "all_status_ok": all(st == 0 for st in statuses),
        "batched_equals_sequential_bitwise": same,
        "mixed_vs_fp64_alone_rel_l2_sample": diffs,
    }


def serve_mode(args, B, W, torch):
    from paper_1611_05677_amd import serving as S
    count = args.requests
    warm = min(200, count // 5)
    trace = W.serving_trace(count=count, rate_hz=args.rate)
    reqs = S.requests_from_trace(trace)
    ex = S.DeviceExecutor(B.FMG_MIXED, "cuda:0", max_inflight=args.inflight)
    srv = S.Server(ex, budget_bytes=64 << 30, max_inflight=args.inflight)
    # resident hierarchies and captured graphs for every shape and nonlinearity
    # are built by a warm-up pass (not timed), as a long-running server would
    warm_reqs = []
    rid = -1
    for dim, (lo, hi) in ((2, (7, 10)), (3, (3, 6))):
        for d in range(lo, hi + 1):
            for kind in W.SERVE_KINDS:
                warm_reqs.append(S.ServedRequest(rid, 0.0, dim, d, kind, 0.0, W.fourier_coefficients(dim, 16, [0, -rid])))
                rid -= 1
    srv.run(warm_reqs)
    torch.cuda.synchronize()
    out = srv.run(reqs)
    torch.cuda.synchronize()
    summ = S.latency_summary(out, skip=warm)
    dofs = sum((4 * 2 ** r.refinements - 1) ** r.dim for r in out[warm:])
    srv.close()
    return {
        "metric": METRIC, "value": dofs / summ["span_s"], "unit": "DOF/s", "n_gpus": 1, "steps": count - warm,
        "warmup": warm, "ms_per_step": 1e3 * summ["span_s"] / max(1, summ["requests"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": SERVE_DESC, "requests": count, "measured_after": warm,
                   "max_inflight": args.inflight, "rate_hz": args.rate},
        "latency_ms_p50": summ["latency_ms_p50"], "latency_ms_p99": summ["latency_ms_p99"],
        "latency_ms_mean": summ["latency_ms_mean"], "solves_per_s": summ["solves_per_s"],
        "all_status_ok": summ["ok"] == summ["requests"], "max_concurrent": srv.max_concurrent,
        "pool": vars(srv.pool.stats),
    }


def roofline_leg(args, B, torch, factory, depth):
    """The dominant kernel alone (same launches as the bench's roofline) and a
    plain device copy of known size, for the counter runs: the copy's
    FETCH_SIZE / WRITE_SIZE against its known bytes calibrate the counters."""
    dim = 3 if factory.startswith("cube") else 2
    H = B.Hierarchy(dim, 4, depth, B.default_options(dim), device="cuda:0")
    roof = roofline_live(B, H, dim, args.workload, args.roof_reps)
    n = 1 << 25                                   # 32 Mi doubles = 256 MiB each way
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    H.close()
    print(json.dumps({"roofline": roof, "copy_bytes_each_way": 8 * n, "copies": 3}), flush=True)


def measure_workload(args, B, W, torch, key, profile=True, only=None):
    """Float64 and mixed solves of one configuration: throughput, latency,
    accuracy gate, per-kernel profile; returns (record, hierarchies, problem)."""
    desc, factory, depth, gkey = WORKLOADS[key]
    golden = json.load(open(GOLDEN))[gkey]
    P = getattr(W, factory)(depth)
    g = torch.from_numpy(P.g_nodes).to("cuda:0")
    log(f"workload {key}: {P.name} n={P.n} DOFs={P.interior_dofs}")
    uc, conv_info = converged_solution(B, torch, P, g, golden)
    modes, hier = {}, {}
    for name, prec in (("fp64", B.FMG_FP64), ("mixed", B.FMG_MIXED)):
        if only and name != only:
            continue
        H, res = run_mode(B, torch, P, g, prec, args.steps, args.warmup, golden, uc)
        modes[name] = res
        hier[name] = H
        log(f"{name}: {res['ms_per_solve']:.3f} ms/solve, {res['dof_per_s'] / 1e9:.3f} GDOF/s, "
            f"p50 {res['latency_ms_p50']:.3f} ms p99 {res['latency_ms_p99']:.3f} ms, "
            f"alg/disc {res['alg_over_disc']:.3f}, gate {res['gate_pass']}")
    if profile:
        for name in modes:
            total_ms, rows = profile_mode(B, hier[name], P, g, torch)
            by_kernel = roofline_from_profile(rows)
            modes[name]["profile_event_ms_total"] = total_ms
            modes[name]["profile_rows_all"] = rows
            modes[name]["profile_ms_by_kernel"] = {k: round(v, 4) for k, v in
                                                   sorted(by_kernel.items(), key=lambda kv: -kv[1])}
    rec = {"workload": desc, "dofs": P.interior_dofs, "levels": P.n_levels,
           "converged_reference": conv_info, "modes": modes}
    for name in modes:
        rec[f"dof_per_s_{name}"] = modes[name]["dof_per_s"]
    if len(modes) == 2:
        rec["mixed_speedup_vs_fp64"] = modes["mixed"]["dof_per_s"] / modes["fp64"]["dof_per_s"]
    return rec, hier, P


EXAMPLES_DESC = ("the paper's Examples 1-3 on (0,1)^3 (Kuhn tetrahedra, coarse 4^3, m = 2, p = 1): "
                 "Ex. 1 f = u^3, u = sin sin sin; Ex. 2 -Lap u - exp(-u) = 1 (no closed form); "
                 "Ex. 3 f = sign(u)|u|^{3/2}, u = sin 2pi x sin 2pi y sin 2pi z; float64, depths 1-6")


def examples_mode(args, B, W, torch):
    """Errors and time per level for the paper's 3D examples: nodal L2 error
    against the exact solution (Ex. 1, 3) or against the next finer level's
    solution injected (Ex. 2), with observed rates, and fine DOF/s per level."""
    depths = list(range(1, args.max_depth + 1))
    out = {}
    for ex, factory in ((1, W.cube_example1), (2, W.cube_example2), (3, W.cube_example3)):
        rows, prev = [], None
        for L in depths:
            P = factory(L)
            g = torch.from_numpy(P.g_nodes).to("cuda:0")
            H = B.Hierarchy(3, 4, L, B.default_options(3), device="cuda:0")
            u = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
            for _ in range(2):
                H.solve_async(g, P.f_kind, P.f_param, u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                H.solve_async(g, P.f_kind, P.f_param, u)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            rep = H.report()
            H.close()
            n = P.n
            un = u.cpu().numpy().reshape((n + 1,) * 3)
            row = {"depth": L, "n": n, "dofs": P.interior_dofs, "ms_per_solve": ms,
                   "dof_per_s": P.interior_dofs / (ms * 1e-3), "status": rep["status"]}
            if P.u_exact_nodes is not None:
                ue = P.u_exact_nodes.reshape((n + 1,) * 3)
                row["err_nodal_l2"] = float(np.sqrt(np.sum((un - ue) ** 2) / n ** 3))
            if ex == 2 and prev is not None:
                # previous (coarser) level's solution against this one at the shared nodes
                pn = prev.shape[0] - 1
                diff = prev - un[::2, ::2, ::2]
                rows[-1]["err_nodal_l2_vs_finer"] = float(np.sqrt(np.sum(diff ** 2) / pn ** 3))
            prev = un
            rows.append(row)
            log(f"example {ex} depth {L}: {ms:.3f} ms, {row['dof_per_s'] / 1e9:.3f} GDOF/s, "
                f"err {row.get('err_nodal_l2', float('nan')):.3e}")
        key = "err_nodal_l2" if ex != 2 else "err_nodal_l2_vs_finer"
        for a, b in zip(rows, rows[1:]):
            if a.get(key) and b.get(key):
                b["rate"] = float(np.log2(a[key] / b[key]))
        out[f"example{ex}"] = rows
    top = out["example1"][-1]
    return {
        "metric": METRIC, "value": top["dof_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": 5, "warmup": 2,
        "ms_per_step": top["ms_per_solve"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": EXAMPLES_DESC, "value_is": "Example 1 at the deepest level"},
        "examples": out,
    }


ELEMENT_DESC = ("element rule: the cube256 problem (3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 6 times, "
                "256^3, 16,581,375 DOFs, -Lap u + u + sin u = g, g manufactured from u = sin sin sin, m = 2, p = 1) "
                "with the L2 pairings (f(u), v) and (g, v) taken by a degree-2 rule on every fine tetrahedron "
                "(4 points), u_h, v_h and g as P1 interpolants, in the linearised load, the augmented problem "
                "and level 1")
# the element-rule quadrature pass (setup excluded) at the finest level
ALU_KERNEL_ELEMENT = ("aug_pass", "fmg_elem.h")


def element_cpu_baseline(W):
    """The element-rule oracle O2 on the host, single thread, on a bounded
    sample: the same manufactured problem two levels coarser (64^3).  One
    untimed solve builds the per-level element rules (the analogue of the
    hierarchy creation); the second is timed."""
    from threadpoolctl import threadpool_limits

    from oracle.nonlinear import Nonlinearity
    from oracle.o2 import Hierarchy as O2H
    from oracle.o2 import Options as O2Options
    from oracle.o2 import fmg as o2_fmg
    S = W.cube_u_plus_sin(4)
    with threadpool_limits(limits=1):
        H = O2H(S.dim, S.coarse_cells, S.refinements)
        opts = O2Options(quadrature="element")
        nl = Nonlinearity(S.f_kind, S.f_param)
        o2_fmg(H, S.g_nodes, nl, opts)
        t0 = time.perf_counter()
        o2_fmg(H, S.g_nodes, nl, opts)
        o2_s = time.perf_counter() - t0
    return {"value": S.interior_dofs / o2_s, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"O2 with the element rule (scipy CSR, the oracle's replica of the FMG scheme): {S.name} "
                      f"({S.interior_dofs} DOFs, the benchmark's problem two levels coarser), one solve "
                      f"{o2_s:.2f} s after an untimed one that builds the element rules",
            "o2_solve_s": o2_s, "o2_dofs": S.interior_dofs, "cpu_model": _cpu_model(),
            "threads_used": "1 (scipy sparse kernels are single-threaded; BLAS pools limited to 1)"}


def element_mode(args, B, W, torch):
    """The element-rule reading (fmg_options.quadrature = FMG_QUAD_ELEMENT) on
    the largest configuration: float64 and mixed throughput and latency, the
    accuracy gate against ubar_h of the same reading (the library's converged
    mode, which the tests match to the element-rule oracle O1), the distance to
    the vertex-rule solution, the float64 ALU roofline of the element
    quadrature pass and the per-kernel profile."""
    depth = 6
    P = W.cube_u_plus_sin(depth)
    g = torch.from_numpy(P.g_nodes).to("cuda:0")
    EL = B.FMG_QUAD_ELEMENT
    if args.only:
        # trace and counter runs: the timed solves of one precision only
        uc = uv = np.zeros(P.g_nodes.shape)
        crep = {"status": None, "extra_steps": None, "last_update_rel": None}
    else:
        Hc = B.Hierarchy(3, 4, depth, B.default_options(3, mode=B.FMG_CONVERGED, quadrature=EL), device="cuda:0")
        uct, crep = Hc.solve(g, P.f_kind, P.f_param)
        Hc.close()
        uc = uct.cpu().numpy()
        Hv = B.Hierarchy(3, 4, depth, B.default_options(3), device="cuda:0")
        uvt, _ = Hv.solve(g, P.f_kind, P.f_param)
        Hv.close()
        uv = uvt.cpu().numpy()
    disc = nodal(P, uc - P.u_exact_nodes)
    stream = torch.cuda.current_stream()
    modes, rows = {}, None
    for name, prec in (("fp64", B.FMG_FP64), ("mixed", B.FMG_MIXED)):
        if args.only and name != args.only:
            continue
        H = B.Hierarchy(3, 4, depth, B.default_options(3, precision=prec, quadrature=EL), device="cuda:0")
        out = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
        for _ in range(args.warmup):
            H.solve_async(g, P.f_kind, P.f_param, out)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
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
        exact_err, alg = nodal(P, u - P.u_exact_nodes), nodal(P, u - uc)
        res = {"dof_per_s": P.interior_dofs / (wall / args.steps), "ms_per_solve": 1e3 * wall / args.steps,
               "latency_ms_p50": percentile(lat, 50), "latency_ms_p99": percentile(lat, 99),
               "status": rep["status"], "newton_iters": rep["newton_iters"], "level1_iters": rep["level1_iters"],
               "err_vs_exact_nodal_l2": exact_err, "disc_nodal_l2": disc, "alg_nodal_l2": alg,
               "alg_over_disc": alg / disc,
               "gate_total_le_1.1disc": bool(exact_err <= 1.1 * disc),
               "gate_alg_le_0.5disc": bool(alg <= 0.5 * disc),
               "vertex_rule_distance_over_disc": nodal(P, u - uv) / disc}
        res["gate_pass"] = bool(res["gate_total_le_1.1disc"] and res["gate_alg_le_0.5disc"] and rep["status"] == 0)
        if name == "fp64" and not args.no_profile:
            total_ms, rows = profile_mode(B, H, P, g, torch)
            res["profile_event_ms_total"] = total_ms
            res["profile_rows"] = sorted(rows, key=lambda r: -r["ms"])[:30]
        H.close()
        modes[name] = res
        log(f"element {name}: {res['ms_per_solve']:.3f} ms/solve, {res['dof_per_s'] / 1e9:.3f} GDOF/s, "
            f"alg/disc {res['alg_over_disc']:.3f}, gate {res['gate_pass']}")
    alu = alu_roofline(rows, "cube256_element", P.n_levels, 3, ALU_KERNEL_ELEMENT) if rows else None
    if args.only:
        return {"only": args.only, "modes": {k: {q: v for q, v in m.items() if q != "profile_rows"}
                                             for k, m in modes.items()}}
    primary = modes["fp64"]
    line = {
        "metric": METRIC, "value": primary["dof_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": primary["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": ELEMENT_DESC, "dofs": P.interior_dofs, "levels": P.n_levels,
                   "precision_of_value": "fp64 (plain)"},
        "latency_ms_p50": primary["latency_ms_p50"], "latency_ms_p99": primary["latency_ms_p99"],
        "gate_pass": primary["gate_pass"],
        "mixed": {k: modes["mixed"][k] for k in ("dof_per_s", "ms_per_solve", "latency_ms_p50",
                                                 "latency_ms_p99", "gate_pass", "alg_over_disc")},
        "mixed_speedup_vs_fp64": modes["mixed"]["dof_per_s"] / primary["dof_per_s"],
        "converged_reference": {"status": crep["status"], "extra_steps": crep["extra_steps"],
                                "last_update_rel": crep["last_update_rel"],
                                "source": "the library's converged mode, element rule"},
        "modes": modes,
        "roofline": alu,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = element_cpu_baseline(W)
    return line


VARIABLE_DESC = ("variable coefficient: 3D unit cube, Kuhn tetrahedra, coarse 4^3 refined 6 times (256^3, "
                 "16,581,375 DOFs); -div(A grad u) + c(x) (u + sin u) = g with A(x) = (1 + s/2) B constant per cell "
                 "(s = sin(pi x) sin(pi y) sin(pi z) at the cell centre, B a fixed symmetric positive definite "
                 "matrix with off-diagonal entries: the 15-point Kuhn stencil), c = 1 + cos(pi x)/2 at the nodes, "
                 "g manufactured from u = s; every level the Galerkin restriction of the finest form; m = 2 V(2,2) "
                 "Chebyshev-weighted cycles, p = 1, float64")
# the weighted Jacobi sweep at the finest level (HBM bound: x, b, the seven
# forward-edge weight planes in, the new iterate out)
VAR_ROOF_KERNEL = ("smooth_var_f64", "fmg_kernels_coef.h")


def variable_cpu_baseline(W):
    """The variable-coefficient oracle O2 on the host, single thread, on a
    bounded sample: the same manufactured problem one level coarser (128^3).
    The Galerkin hierarchy (the analogue of fmg_create_hierarchy plus
    fmg_set_coefficients; about a minute and 14 GB) is built untimed; the
    median of three solves is reported."""
    from threadpoolctl import threadpool_limits

    from oracle.nonlinear import Nonlinearity
    from oracle.o2 import Hierarchy as O2H
    from oracle.o2 import fmg as o2_fmg
    S = W.variable_coefficient("cube128_var", 3, 4, 5, W.F_U_PLUS_SIN)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        H = O2H(S.dim, S.coarse_cells, S.refinements, coef=S.coef_cells)
        build_s = time.perf_counter() - t0
        nl = Nonlinearity(S.f_kind, S.f_param)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            o2_fmg(H, S.g_nodes, nl, f_weight=S.f_weight_nodes)
            times.append(time.perf_counter() - t0)
        o2_s = float(np.median(times))
    return {"value": S.interior_dofs / o2_s, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"O2 with the coefficients (scipy CSR, the oracle's replica of the FMG scheme): {S.name} "
                      f"({S.interior_dofs} DOFs, the benchmark's problem one level coarser), median of 3 "
                      f"solves {o2_s:.3f} s; Galerkin hierarchy {build_s:.1f} s not timed",
            "o2_solve_s": o2_s, "o2_dofs": S.interior_dofs, "hierarchy_s": build_s, "cpu_model": _cpu_model(),
            "threads_used": "1 (scipy sparse kernels are single-threaded; BLAS pools limited to 1)"}


def variable_mode(args, B, W, torch):
    """The variable-coefficient operator (fmg_options.coefficients =
    FMG_COEF_VARIABLE) on the largest configuration: float64 throughput and
    latency of the solve (the operator set once beforehand, its setup timed
    on its own), the accuracy gate against ubar_h of the same operator (the
    library's converged mode, which the tests match to the oracle O1), the
    HBM roofline of the weighted sweep and the per-kernel profile."""
    depth = 6
    P = W.variable_coefficient("cube256_var", 3, 4, depth, W.F_U_PLUS_SIN)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")   # noqa: E731
    g, c, coef = dev(P.g_nodes), dev(P.f_weight_nodes), dev(P.coef_cells)
    VAR = B.FMG_COEF_VARIABLE
    if args.roofline_only:
        # counter runs: the weighted sweep alone (as timed below) and a plain
        # 256 MiB device copy that calibrates FETCH_SIZE / WRITE_SIZE
        H = B.Hierarchy(3, 4, depth, B.default_options(3, coefficients=VAR), device="cuda:0")
        H.set_coefficients(coef)
        ms, nbytes = B.time_level_kernel(H, VAR_ROOF_KERNEL[0], H.levels, args.roof_reps)
        n = 1 << 25
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        H.close()
        return {"roofline_only": VAR_ROOF_KERNEL[0], "avg_launch_us": ms * 1e3, "bytes_per_launch": nbytes,
                "copy_bytes_each_way": 8 * n, "copies": 3}
    if args.only:
        uc = np.zeros(P.g_nodes.shape)
        crep = {"status": None, "extra_steps": None, "last_update_rel": None}
    else:
        Hc = B.Hierarchy(3, 4, depth, B.default_options(3, mode=B.FMG_CONVERGED, coefficients=VAR), device="cuda:0")
        Hc.set_coefficients(coef)
        uct, crep = Hc.solve(g, P.f_kind, P.f_param, c=c)
        Hc.close()
        uc = uct.cpu().numpy()
    disc = nodal(P, uc - P.u_exact_nodes)
    stream = torch.cuda.current_stream()
    H = B.Hierarchy(3, 4, depth, B.default_options(3, coefficients=VAR), device="cuda:0")
    setup_ms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        H.set_coefficients(coef)
        b.record(stream)
        torch.cuda.synchronize()
        setup_ms.append(a.elapsed_time(b))
    out = torch.empty(H.nodes(), dtype=torch.float64, device="cuda:0")
    for _ in range(args.warmup):
        H.solve_async(g, P.f_kind, P.f_param, out, c=c)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        H.solve_async(g, P.f_kind, P.f_param, out, c=c)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in ev]
    rep = H.report()
    u = out.cpu().numpy()
    exact_err, alg = nodal(P, u - P.u_exact_nodes), nodal(P, u - uc)
    res = {"dof_per_s": P.interior_dofs / (wall / args.steps), "ms_per_solve": 1e3 * wall / args.steps,
           "latency_ms_p50": percentile(lat, 50), "latency_ms_p99": percentile(lat, 99),
           "status": rep["status"], "newton_iters": rep["newton_iters"], "level1_iters": rep["level1_iters"],
           "err_vs_exact_nodal_l2": exact_err, "disc_nodal_l2": disc, "alg_nodal_l2": alg,
           "alg_over_disc": alg / disc if disc > 0 else None,
           "gate_total_le_1.1disc": bool(exact_err <= 1.1 * disc),
           "gate_alg_le_0.5disc": bool(alg <= 0.5 * disc)}
    res["gate_pass"] = bool(res["gate_total_le_1.1disc"] and res["gate_alg_le_0.5disc"] and rep["status"] == 0)
    log(f"variable fp64: {res['ms_per_solve']:.3f} ms/solve, {res['dof_per_s'] / 1e9:.3f} GDOF/s, "
        f"setup {min(setup_ms):.2f} ms, alg/disc {res['alg_over_disc']}, gate {res['gate_pass']}")
    rows = None
    if not args.no_profile:
        total_ms, rows = profile_mode(B, H, P, g, torch, c)
        res["profile_event_ms_total"] = total_ms
        res["profile_rows"] = sorted(rows, key=lambda r: -r["ms"])[:30]
    name, fname = VAR_ROOF_KERNEL
    ms, nbytes = B.time_level_kernel(H, name, H.levels, args.roof_reps)
    achieved = nbytes / (ms * 1e-3) / 1e9
    e = _counter_entry(TRAFFIC_FILE, name, "cube256_var", fname)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": e["hbm_bytes_per_launch"] if e else None,
            "kernel": name, "level": H.levels, "launches_timed": args.roof_reps, "avg_launch_us": ms * 1e3,
            "bytes_per_launch": nbytes,
            "bytes_model": "8 B x 10 N: read x, b and the seven forward-edge weight planes, write the new "
                           "iterate, N interior nodes of the level",
            "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if e else None}
    H.close()
    if args.only:
        return {"only": args.only, "modes": {"fp64": {q: v for q, v in res.items() if q != "profile_rows"}},
                "roofline": roof}
    line = {
        "metric": METRIC, "value": res["dof_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": VARIABLE_DESC, "dofs": P.interior_dofs, "levels": P.n_levels,
                   "precision_of_value": "fp64 (plain; the variable operator runs in float64 only)"},
        "latency_ms_p50": res["latency_ms_p50"], "latency_ms_p99": res["latency_ms_p99"],
        "gate_pass": res["gate_pass"],
        "coef_setup_ms": {"min": min(setup_ms), "all": setup_ms,
                          "what": "fmg_set_coefficients: per-simplex means on every level, forward-edge "
                                  "weights, A_1 and its inverse (once per coefficient field, outside the solve)"},
        "converged_reference": {"status": crep["status"], "extra_steps": crep["extra_steps"],
                                "last_update_rel": crep["last_update_rel"],
                                "source": "the library's converged mode, same operator"},
        "modes": {"fp64": res},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = variable_cpu_baseline(W)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 2D 2048^2 record")
    ap.add_argument("--workload", default="cube256",
                    choices=sorted(WORKLOADS) + ["batch64", "serve", "examples", "element", "variable"])
    ap.add_argument("--max-depth", type=int, default=6, help="examples: deepest refinement")
    ap.add_argument("--requests", type=int, default=4000, help="serve: requests in the trace")
    ap.add_argument("--inflight", type=int, default=8, help="serve: concurrent solves")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: mean arrival rate (requests/s)")
    ap.add_argument("--roof-reps", type=int, default=200, help="launches timed for the roofline kernel")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline leg (dominant kernel + a reference copy), for counter runs")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="time one precision only (for traces and counter runs); no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver runs on a single "
              "device, and sharding a solve or a request stream over several GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)

    from paper_1611_05677_amd import build as build_mod
    if not os.path.exists(build_mod.LIB):
        build_mod.build()
    import torch

    from paper_1611_05677_amd import binding as B
    from paper_1611_05677_amd import workloads as W

    if args.workload in ("batch64", "serve", "examples", "element", "variable"):
        mode = {"batch64": batch_mode, "serve": serve_mode, "examples": examples_mode,
                "element": element_mode, "variable": variable_mode}[args.workload]
        line = mode(args, B, W, torch)
        print(json.dumps(line), flush=True)
        return
    desc, factory, depth, gkey = WORKLOADS[args.workload]
    if args.roofline_only:
        roofline_leg(args, B, torch, factory, depth)
        return
    if args.only:
        rec, hier, P = measure_workload(args, B, W, torch, args.workload, profile=not args.no_profile,
                                        only=args.only)
        for H in hier.values():
            H.close()
        log(json.dumps({k: v for k, v in rec.items() if k != "modes"}))
        return
    rec, hier, P = measure_workload(args, B, W, torch, args.workload, profile=not args.no_profile)
    modes = rec["modes"]
    roof = roofline_live(B, hier["fp64"], P.dim, args.workload, args.roof_reps)
    log(f"roofline: {roof['kernel']} level {roof['level']}: {roof['avg_launch_us']:.2f} us/launch, "
        f"{roof['achieved']:.0f} GB/s = {100 * roof['frac']:.1f}% of {HBM_PEAK_GBS:.0f} GB/s")
    alu = None
    if not args.no_profile:
        alu = alu_roofline(modes["fp64"]["profile_rows_all"], args.workload, P.n_levels, P.dim)
        if alu:
            log(f"alu roofline: {alu['kernel']} level {alu['level']}: {alu['avg_launch_us']:.2f} us/launch, "
                f"{alu['achieved'] or float('nan'):.2f} TFLOP/s")
    for m in modes.values():
        if "profile_rows_all" in m:
            m["profile_rows"] = sorted(m.pop("profile_rows_all"), key=lambda r: -r["ms"])[:40]
    for H in hier.values():
        H.close()
    primary = modes["fp64"]
    line = {
        "metric": METRIC, "value": primary["dof_per_s"], "unit": "DOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": primary["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "dofs": P.interior_dofs, "levels": P.n_levels,
                   "precision_of_value": "fp64 (plain)"},
        "latency_ms_p50": primary["latency_ms_p50"], "latency_ms_p99": primary["latency_ms_p99"],
        "gate_pass": primary["gate_pass"],
        "mixed": {k: modes["mixed"][k] for k in ("dof_per_s", "ms_per_solve", "latency_ms_p50",
                                                 "latency_ms_p99", "gate_pass", "alg_over_disc")},
        "mixed_speedup_vs_fp64": rec["mixed_speedup_vs_fp64"],
        "converged_reference": rec["converged_reference"],
        "modes": modes,
        "roofline": roof,
        "alu_roofline": alu,
    }
    sec = SECONDARY.get(args.workload)
    if sec and not args.no_secondary:
        srec, shier, SP = measure_workload(args, B, W, torch, sec, profile=False)
        sroof = roofline_live(B, shier["fp64"], SP.dim, sec, args.roof_reps)
        for H in shier.values():
            H.close()
        for m in srec["modes"].values():
            for k in ("profile_rows_all",):
                m.pop(k, None)
        srec["effective_roofline"] = sroof
        line["secondary"] = {sec: srec}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        line["cpu_baseline"] = cpu_baseline(P, W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
