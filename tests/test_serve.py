"""Serving loop logic on the CPU (fake executor): admission by memory,
grouping of same-semiring requests, isolation of failures, FIFO mode."""
import threading
import time

from paper_2111_09947_amd.serve import Request, Server, percentiles, run_trace


class FakeExec:
    def __init__(self, delay=0.002, fail_on=None):
        self.delay = delay
        self.fail_on = fail_on or set()
        self.lock = threading.Lock()
        self.groups = []
        self.mem = 0
        self.max_mem = 0
        self.active = 0
        self.max_active = 0

    def __call__(self, slot, group, report=None):
        with self.lock:
            self.groups.append([r.rid for r in group])
            self.mem += sum(r.mem_bytes for r in group)
            self.max_mem = max(self.max_mem, self.mem)
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        time.sleep(self.delay)
        with self.lock:
            self.mem -= sum(r.mem_bytes for r in group)
            self.active -= 1
        if any(r.rid in self.fail_on for r in group):
            raise RuntimeError("injected failure")
        for r in group:
            r.result = ("ok", r.rid)


def _mk(i, sr=None, est=100):
    return Request(rid=i, semiring=sr or ("a" if i % 2 else "b"), operands=None, mem_bytes=est)


def test_all_complete_and_latency_positive():
    ex = FakeExec()
    srv = Server(ex, slots=3, max_batch=4)
    reqs = run_trace(srv, lambda i: _mk(i), [0.001 * i for i in range(40)])
    assert all(r.done.is_set() and r.error is None and r.result == ("ok", r.rid) for r in reqs)
    assert all(r.latency > 0 for r in reqs)
    assert ex.max_active <= 3
    p = percentiles([r.latency for r in reqs])
    assert p["p50"] <= p["p99"]


def test_groups_share_a_semiring():
    ex = FakeExec(delay=0.01)
    srv = Server(ex, slots=1, max_batch=8)
    reqs = run_trace(srv, lambda i: _mk(i), [0.0] * 30)
    by = {r.rid: r.semiring for r in reqs}
    for g in ex.groups:
        assert len({by[x] for x in g}) == 1
        assert len(g) <= 8
    assert any(len(g) > 1 for g in ex.groups)  # continuous batching happened


def test_memory_budget_is_respected_and_oversize_rejected():
    ex = FakeExec(delay=0.005)
    srv = Server(ex, slots=4, max_batch=4, mem_budget=1000)
    sizes = [300, 400, 5000, 200, 900, 100, 600]
    reqs = run_trace(srv, lambda i: _mk(i, "a", sizes[i]), [0.0] * len(sizes))
    assert ex.max_mem <= 1000
    big = reqs[2]
    assert big.error and "budget" in big.error
    assert all(r.error is None for k, r in enumerate(reqs) if k != 2)


def test_failure_is_isolated():
    ex = FakeExec(fail_on={3})
    srv = Server(ex, slots=2, max_batch=1)
    reqs = run_trace(srv, lambda i: _mk(i), [0.001 * i for i in range(10)])
    assert reqs[3].error and "injected" in reqs[3].error
    assert all(r.error is None for r in reqs if r.rid != 3)


def test_fifo_mode_runs_one_at_a_time_in_order():
    ex = FakeExec(delay=0.001)
    srv = Server(ex, slots=4, max_batch=8, continuous=False)
    run_trace(srv, lambda i: _mk(i), [0.0] * 12)
    assert ex.max_active == 1
    assert [g for g in ex.groups] == [[i] for i in range(12)]


def test_device_pool_first_fit_and_merging():
    """The shared budget buffer: contiguous reservations in 256-byte granules,
    first fit, freed regions merged with their neighbours, pieces carved in
    order, a piece beyond the region served from its own block."""
    import torch
    from paper_2111_09947_amd.serve import DevicePool
    pool = DevicePool(4096, torch.device("cpu"))
    a, b, c = pool.reserve(1000), pool.reserve(1024), pool.reserve(1500)
    assert (a.off, a.size, b.off, c.off, c.size) == (0, 1024, 1024, 2048, 1536)
    assert pool.reserve(1024) is None and pool.largest_free() == 512
    x, y = a.alloc(10), a.alloc(300)
    assert y.data_ptr() - x.data_ptr() == 256 and x.data_ptr() == pool.buf.data_ptr()
    z = a.alloc(1000)  # beyond the region
    assert a.overflow == 1024 and not (pool.buf.data_ptr() <= z.data_ptr() < pool.buf.data_ptr() + 4096)
    pool.release(b)
    assert pool.free == [[1024, 1024], [3584, 512]]
    pool.release(a)
    assert pool.free == [[0, 2048], [3584, 512]]
    d = pool.reserve(2048)
    assert d.off == 0
    pool.release(c)
    pool.release(d)
    assert pool.free == [[0, 4096]]


def test_pool_admission_with_margins():
    """With a pool's margins a group's reservation exceeds its products'
    bytes; the scheduler still never holds more than the budget."""
    from paper_2111_09947_amd.serve import Budget

    class Margined(Budget):
        def margin(self, count):
            return 50 + 10 * count

    ex = FakeExec(delay=0.005)
    srv = Server(ex, slots=3, max_batch=3, mem_budget=1000, memory=Margined(1000))
    sizes = [300, 400, 200, 900, 100, 600, 950]
    reqs = run_trace(srv, lambda i: _mk(i, "a", sizes[i]), [0.0] * len(sizes))
    assert ex.max_mem <= 1000
    assert reqs[6].error and "budget" in reqs[6].error  # 950 + 60 > 1000
    assert all(r.error is None for r in reqs[:6])
    assert srv.memory.in_use == 0


def test_heavy_requests_run_alone():
    ex = FakeExec(delay=0.002)
    srv = Server(ex, slots=1, max_batch=8, group_work_max=100)
    work = [10, 500, 20, 30, 900, 40, 50, 60]

    def mk(i):
        r = _mk(i, "a")
        r.work = work[i]
        return r
    run_trace(srv, mk, [0.0] * len(work))
    for g in ex.groups:
        assert len(g) == 1 or all(work[x] <= 100 for x in g)
    assert [1] in ex.groups and [4] in ex.groups
    assert any(len(g) > 1 for g in ex.groups)
