"""Host logic of the served-solve loop (admission by footprint, slots,
first-come-first-served order, release of idle hierarchies), driven by a
simulated executor and clock: no GPU involved."""
import pytest

from paper_1611_05677_amd.serving import HierarchyPool, ServedRequest, Server, latency_summary


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Hierarchies are integers; a solve of shape (dim, depth) takes
    `service[key]` seconds of simulated time from its launch."""

    def __init__(self, clock, service, nbytes, dt=1e-4):
        self.clock, self.service, self.nbytes, self.dt = clock, service, nbytes, dt
        self.next_id = 0
        self.live = set()
        self.created_keys = []

    def footprint(self, key):
        return self.nbytes[key]

    def create(self, key):
        self.next_id += 1
        self.live.add(self.next_id)
        self.created_keys.append(key)
        return self.next_id

    def destroy(self, h):
        self.live.remove(h)

    def launch(self, h, slot, r):
        assert h in self.live
        return (self.clock() + self.service[r.key], r.rid)

    def done(self, tok):
        return self.clock() >= tok[0]

    def finish(self, h, slot, tok):
        return 0, tok[1]

    def idle(self):
        self.clock.t += self.dt


def make(reqs_spec):
    return [ServedRequest(i, t, d, L, 2) for i, (t, d, L) in enumerate(reqs_spec)]


def test_all_requests_complete_in_arrival_order():
    clk = Clock()
    ex = FakeExecutor(clk, {(2, 7): 0.002, (3, 4): 0.003}, {(2, 7): 100, (3, 4): 100})
    reqs = make([(0.001 * i, 2 if i % 2 else 3, 7 if i % 2 else 4) for i in range(30)])
    srv = Server(ex, budget_bytes=10_000, max_inflight=4, keep_results=True, clock=clk)
    out = srv.run(reqs)
    assert all(r.t_done >= r.arrival_s + ex.service[r.key] - 1e-12 for r in out)
    admits = [r.t_admit for r in out]
    assert admits == sorted(admits)                      # first come, first served
    assert [r.result for r in out] == [r.rid for r in out]
    assert 1 < srv.max_concurrent <= 4                   # overlapping, within the slots
    s = latency_summary(out)
    assert s["requests"] == 30 and s["ok"] == 30 and s["latency_ms_p50"] >= 2.0


def test_budget_bounds_resident_memory_and_concurrency():
    clk = Clock()
    ex = FakeExecutor(clk, {(2, 7): 0.005}, {(2, 7): 400})
    reqs = make([(0.0, 2, 7)] * 10)
    srv = Server(ex, budget_bytes=1000, max_inflight=8, clock=clk)
    out = srv.run(reqs)
    assert all(r.t_done > 0 for r in out)
    assert srv.pool.stats.peak_bytes <= 1000
    assert srv.max_concurrent == 2                       # two 400-byte hierarchies fit
    assert srv.pool.stats.created == 2                   # then they are reused


def test_idle_hierarchies_of_other_shapes_are_released_when_memory_is_short():
    clk = Clock()
    ex = FakeExecutor(clk, {(2, 7): 0.001, (2, 10): 0.001}, {(2, 7): 600, (2, 10): 900})
    reqs = make([(0.0, 2, 7), (0.01, 2, 10), (0.02, 2, 7)])
    srv = Server(ex, budget_bytes=1000, max_inflight=2, clock=clk)
    srv.run(reqs)
    assert ex.created_keys == [(2, 7), (2, 10), (2, 7)]
    assert srv.pool.stats.released == 2
    assert srv.pool.resident <= 1000


def test_sequential_requests_reuse_one_resident_hierarchy():
    clk = Clock()
    ex = FakeExecutor(clk, {(3, 5): 0.001}, {(3, 5): 10})
    reqs = make([(0.01 * i, 3, 5) for i in range(8)])
    srv = Server(ex, budget_bytes=100, max_inflight=4, clock=clk)
    srv.run(reqs)
    assert srv.pool.stats.created == 1
    srv.close()
    assert not ex.live


def test_request_larger_than_budget_is_rejected():
    clk = Clock()
    ex = FakeExecutor(clk, {(2, 10): 0.001}, {(2, 10): 5000})
    pool = HierarchyPool(ex, 1000)
    with pytest.raises(ValueError):
        pool.acquire((2, 10))
