"""Served solves: a request loop over the C ABI with continuous batching.

* Hierarchies stay resident on the device between requests, pooled by shape
  (dimension, depth); a request takes a free hierarchy of its shape or a new
  one is created, and admission is decided by device-memory footprint
  (fmg_workspace_bytes plus the output array) against a budget; idle
  hierarchies of other shapes are released when memory is short.
* Requests that arrive while others run are admitted as soon as an
  execution slot and memory are free (no batch boundary to wait for).  Every
  admitted request runs on its own HIP stream, so the solves of different
  requests overlap on the device; each solve is one launch of its
  hierarchy's captured graph.
* Latency = time the completion is observed - scheduled arrival time (open
  loop: queueing included).

The pool and the loop take their device operations from an executor object,
so the host logic is testable without a GPU (see the CPU tests).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServedRequest:
    rid: int
    arrival_s: float
    dim: int
    refinements: int
    f_kind: int
    f_param: float = 0.0
    coef: np.ndarray | None = None        # Fourier coefficients of the load
    # filled in by the server
    t_admit: float = -1.0
    t_done: float = -1.0
    status: int = -1
    result: object = None
    concurrent_at_launch: int = 0

    @property
    def key(self):
        return (self.dim, self.refinements)

    @property
    def latency_s(self) -> float:
        return self.t_done - self.arrival_s


@dataclass
class PoolStats:
    created: int = 0
    released: int = 0
    peak_bytes: int = 0
    refused: int = 0


class HierarchyPool:
    """Resident hierarchies by shape, under a device-memory budget."""

    def __init__(self, executor, budget_bytes: int):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.free = collections.defaultdict(collections.deque)   # key -> idle handles
        self.idle_order = collections.OrderedDict()               # handle -> key, LRU first
        self.bytes_of = {}                                        # handle -> footprint
        self.resident = 0
        self.stats = PoolStats()

    def footprint(self, key) -> int:
        return self.ex.footprint(key)

    def acquire(self, key):
        """A hierarchy of shape `key`, or None when it does not fit yet."""
        q = self.free[key]
        if q:
            h = q.popleft()
            self.idle_order.pop(h, None)
            return h
        need = self.footprint(key)
        if need > self.budget:
            raise ValueError(f"request shape {key} needs {need} bytes, above the budget {self.budget}")
        # release idle hierarchies (least recently used first) until it fits
        while self.resident + need > self.budget and self.idle_order:
            h, k = self.idle_order.popitem(last=False)
            self.free[k].remove(h)
            self._destroy(h)
        if self.resident + need > self.budget:
            self.stats.refused += 1
            return None
        h = self.ex.create(key)
        self.bytes_of[h] = need
        self.resident += need
        self.stats.created += 1
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.resident)
        return h

    def release(self, h, key):
        self.free[key].append(h)
        self.idle_order[h] = key

    def _destroy(self, h):
        self.resident -= self.bytes_of.pop(h)
        self.stats.released += 1
        self.ex.destroy(h)

    def close(self):
        for h in list(self.idle_order):
            self._destroy(h)
        self.idle_order.clear()
        self.free.clear()


class Server:
    """Open-loop request loop: arrivals, admission, launch, completion."""

    def __init__(self, executor, budget_bytes: int = 64 << 30, max_inflight: int = 8,
                 keep_results: bool = False, clock=time.perf_counter):
        self.ex = executor
        self.pool = HierarchyPool(executor, budget_bytes)
        self.max_inflight = int(max_inflight)
        self.keep_results = keep_results
        self.clock = clock
        self.max_concurrent = 0

    def run(self, requests: list[ServedRequest], time_scale: float = 1.0) -> list[ServedRequest]:
        """Serve `requests` (sorted by arrival) in real time; returns them with
        their admission / completion times (seconds from the start)."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        waiting = collections.deque()
        inflight = []                       # (request, handle, slot token)
        slots = list(range(self.max_inflight))
        i = 0
        t0 = self.clock()
        while i < len(reqs) or waiting or inflight:
            now = (self.clock() - t0) / time_scale
            while i < len(reqs) and reqs[i].arrival_s <= now:
                waiting.append(reqs[i])
                i += 1
            progressed = False
            # completions
            still = []
            for r, h, slot, tok in inflight:
                if self.ex.done(tok):
                    r.t_done = (self.clock() - t0) / time_scale
                    r.status, out = self.ex.finish(h, slot, tok)
                    if self.keep_results:
                        r.result = out
                    self.pool.release(h, r.key)
                    slots.append(slot)
                    progressed = True
                else:
                    still.append((r, h, slot, tok))
            inflight = still
            # admissions, first come first served
            while waiting and slots:
                r = waiting[0]
                h = self.pool.acquire(r.key)
                if h is None:
                    break                   # memory full: wait for a release
                waiting.popleft()
                slot = slots.pop()
                r.t_admit = (self.clock() - t0) / time_scale
                r.concurrent_at_launch = len(inflight)
                tok = self.ex.launch(h, slot, r)
                inflight.append((r, h, slot, tok))
                self.max_concurrent = max(self.max_concurrent, len(inflight))
                progressed = True
            if not progressed:
                self.ex.idle()
        return reqs

    def close(self):
        self.pool.close()


class DeviceExecutor:
    """Device side of the server: hierarchies, streams and solves through the C ABI."""

    def __init__(self, precision: int, device: str = "cuda:0", coarse_cells: int = 4, max_inflight: int = 8,
                 options=None):
        import torch

        from . import binding as B
        self.B, self.torch = B, torch
        self.precision = precision
        self.device = device
        self.coarse_cells = coarse_cells
        self.options = options or {}
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_inflight)]

    def opts(self, dim):
        return self.B.default_options(dim, precision=self.precision, **self.options)

    def footprint(self, key) -> int:
        dim, depth = key
        n = self.coarse_cells * 2 ** depth
        return self.B.workspace_bytes(dim, self.coarse_cells, depth, self.opts(dim)) + 16 * (n + 1) ** dim

    def create(self, key):
        dim, depth = key
        return self.B.Hierarchy(dim, self.coarse_cells, depth, self.opts(dim), device=self.device)

    def destroy(self, h):
        h.close()

    def launch(self, h, slot, r: ServedRequest):
        torch = self.torch
        from . import workloads as W
        st = self.streams[slot]
        with torch.cuda.stream(st):
            g = W.fourier_load_device(r.coef, h.n, self.device)
            out = torch.empty(h.nodes(), dtype=torch.float64, device=self.device)
            h.solve_async(g, r.f_kind, r.f_param, out, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, out, g)

    def done(self, tok) -> bool:
        return tok[0].query()

    def finish(self, h, slot, tok):
        rep = h.report(stream=self.streams[slot])
        return rep["status"], tok[1]

    def idle(self):
        time.sleep(5e-5)


def latency_summary(reqs: list[ServedRequest], skip: int = 0) -> dict:
    done = [r for r in reqs[skip:] if r.t_done >= 0]
    lat = np.array([r.latency_s for r in done]) * 1e3
    span = max(r.t_done for r in done) - min(r.arrival_s for r in done) if done else 0.0
    return {"requests": len(done), "ok": int(sum(r.status == 0 for r in done)),
            "latency_ms_p50": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if len(lat) else None,
            "latency_ms_mean": float(lat.mean()) if len(lat) else None,
            "solves_per_s": len(done) / span if span > 0 else None,
            "span_s": span}


def requests_from_trace(trace, modes: int = 16) -> list[ServedRequest]:
    """Served requests from an arrival trace (coefficients of each load drawn
    from the request's own seed)."""
    from . import workloads as W
    return [ServedRequest(t.rid, t.arrival_s, t.dim, t.refinements, t.f_kind, 0.0,
                          W.fourier_coefficients(t.dim, modes, t.seed)) for t in trace]
