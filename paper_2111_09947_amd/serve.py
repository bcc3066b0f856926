"""Serving loop for masked products: requests arrive over time, are admitted
while execution slots and device memory allow, and run concurrently on the
GPU (continuous batching).

Design
  - Operands stay resident on the device; a request names them and a
    semiring.
  - A scheduler thread owns the waiting queue. Whenever an execution slot is
    free it takes the oldest waiting request and, in continuous mode, the
    other waiting requests with the same semiring that still fit the memory
    budget (up to max_batch), and hands the group to the slot.
  - Each slot is a worker thread with its own HIP stream (default priority).
    A group of one runs as a single-product plan, a larger group as one batch
    (one launch per kernel bin for all its products). Slots overlap on the
    device.
  - Admission is by memory: a group runs only when its device bytes can be
    reserved from the budget; otherwise it waits. The bytes are the
    library's own sizes for each product (plan workspace, execution
    workspace and the output at its upper bound: product_bytes), taken once
    per resident operand set, plus a margin per group for a batch's tables.
    With the GPU executor the budget is one device buffer shared by all
    slots (DevicePool): a group reserves a contiguous region of it, every
    workspace and every output that is not kept is carved from that region,
    and the region returns to the pool when the group's stream has finished.
    The accounting is then the memory itself, and serving allocates no
    device memory per request. A request that alone exceeds the budget, or
    whose execution raises, completes with an error and the loop keeps
    serving.
  - Latency is measured from the request's arrival time to the moment its
    group's stream has finished (the worker synchronizes its own stream).

The executor is pluggable (CPU tests drive the scheduler with a fake one).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Any, Callable, Deque, Dict, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    semiring: str
    operands: Any               # (A, B, M, complement) for the GPU executor
    mem_bytes: int = 0          # device bytes the product needs (admission)
    work: int = 0               # products of the request (grouping: heavy requests run alone)
    t_arrival: float = 0.0      # perf_counter() time of arrival
    t_start: float = 0.0
    t_done: float = 0.0
    result: Any = None
    keep: bool = False          # keep the result (otherwise dropped after completion)
    error: Optional[str] = None
    region: Any = None          # the group's memory reservation while it runs
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def product_info(A, B, M, complement: bool, semiring: str):
    """(device bytes, products) of one product in the library. The bytes are
    its plan workspace, its execution workspace and its output (row
    pointers, and column indices and values at the upper bound), as the
    library's size queries give them. Runs the row analysis once (one plan
    creation)."""
    from . import Plan, out_dtype
    with Plan(A, B, M, complement=complement, semiring=semiring) as p:
        width = out_dtype(semiring).itemsize
        return (p.plan_workspace_bytes + p.workspace_bytes + 8 * (p.nrows + 1)
                + max(p.upper_bound, 1) * (4 + width)), int(p.products)


def product_bytes(A, B, M, complement: bool, semiring: str) -> int:
    """The device bytes of product_info."""
    return product_info(A, B, M, complement, semiring)[0]


class Budget:
    """Memory accounting by a counter, with no memory behind it: a
    reservation is its byte count, held until release."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.in_use = 0

    def margin(self, count: int) -> int:
        return 0

    def largest_free(self) -> int:
        return self.capacity - self.in_use

    def reserve(self, nbytes: int):
        if nbytes > self.largest_free():
            return None
        self.in_use += nbytes
        return [nbytes]

    def adjust(self, handle, actual: int):
        """The group's real bytes (a batch's tables): the accounting follows."""
        self.in_use += int(actual) - handle[0]
        handle[0] = int(actual)

    def release(self, handle):
        self.in_use -= handle[0]


class Server:
    def __init__(self, executor: Callable[[int, List[Request]], None], slots: int = 4, max_batch: int = 8,
                 mem_budget: int = 64 << 30, continuous: bool = True, memory=None,
                 group_work_max: Optional[int] = None):
        """`memory`: the budget's accounting (reserve / release); default:
        the executor's own pool when it has one (make_memory), else a
        counter. `group_work_max`: requests with more work (products) than
        this run alone and are never grouped (None: no limit); a group then
        gathers only the light requests, for which one batch saves launches
        and synchronizations, while a heavy one fills the GPU by itself."""
        self.executor = executor
        self.slots = slots if continuous else 1
        self.max_batch = max_batch if continuous else 1
        self.mem_budget = mem_budget
        self.continuous = continuous
        self.group_work_max = group_work_max
        if memory is None:
            make = getattr(executor, "make_memory", None)
            memory = make(mem_budget) if make is not None else Budget(mem_budget)
        self.memory = memory
        self._queue: Deque[Request] = collections.deque()
        self._cv = threading.Condition()
        self._free_slots = list(range(self.slots))
        self._running = False
        self._threads: List[threading.Thread] = []
        self._work: Dict[int, Deque[List[Request]]] = {s: collections.deque() for s in range(self.slots)}
        self.completed: List[Request] = []

    def group_bytes(self, reqs) -> int:
        """The reservation of a group: its products' bytes plus the memory's
        margin (a batch's tables, alignment)."""
        return sum(r.mem_bytes for r in reqs) + self.memory.margin(len(reqs))

    # ---- public API
    def start(self):
        self._running = True
        t = threading.Thread(target=self._schedule, daemon=True)
        t.start()
        self._threads.append(t)
        for s in range(self.slots):
            w = threading.Thread(target=self._worker, args=(s,), daemon=True)
            w.start()
            self._threads.append(w)

    def submit(self, req: Request) -> Request:
        if not req.t_arrival:
            req.t_arrival = time.perf_counter()
        with self._cv:
            self._queue.append(req)
            self._cv.notify_all()
        return req

    def stop(self):
        with self._cv:
            self._running = False
            self._cv.notify_all()
        for t in self._threads:
            t.join(timeout=30)

    # ---- scheduler
    def _pick_group(self) -> List[Request]:
        """Oldest request first; then same-semiring requests in arrival order
        while the group's bytes can still be reserved; the reservation is
        taken here (under the lock) and attached to the group's requests."""
        head = self._queue[0]
        if self.group_bytes([head]) > self.mem_budget:
            self._queue.popleft()
            head.error = "request exceeds the memory budget"
            head.t_done = time.perf_counter()
            head.done.set()
            self.completed.append(head)
            return []
        room = self.memory.largest_free()
        if self.group_bytes([head]) > room:
            return []  # wait for memory
        group = [self._queue.popleft()]
        light = self.group_work_max is None or head.work <= self.group_work_max
        if self.continuous and light:
            keep: Deque[Request] = collections.deque()
            while self._queue and len(group) < self.max_batch:
                r = self._queue.popleft()
                if (r.semiring == head.semiring and (self.group_work_max is None or r.work <= self.group_work_max)
                        and self.group_bytes(group + [r]) <= room):
                    group.append(r)
                else:
                    keep.append(r)
            keep.extend(self._queue)
            self._queue = keep
        handle = self.memory.reserve(self.group_bytes(group))
        if handle is None:  # cannot happen below the largest free block; wait rather than fail
            self._queue.extendleft(reversed(group))
            return []
        for r in group:
            r.region = handle
        return group

    def _schedule(self):
        while True:
            with self._cv:
                while self._running and not (self._queue and self._free_slots):
                    self._cv.wait(timeout=0.05)
                if not self._running:
                    return
                group = self._pick_group()
                if not group:
                    if self._queue and self.group_bytes([self._queue[0]]) <= self.mem_budget:
                        self._cv.wait(timeout=0.01)  # memory is held by running groups
                    continue
                slot = self._free_slots.pop(0)
                self._work[slot].append(group)
                self._cv.notify_all()

    def _worker(self, slot: int):
        while True:
            with self._cv:
                while self._running and not self._work[slot]:
                    self._cv.wait(timeout=0.05)
                if not self._running and not self._work[slot]:
                    return
                group = self._work[slot].popleft()
            t0 = time.perf_counter()
            for r in group:
                r.t_start = t0
            handle = group[0].region

            def report(actual: int):
                """The executor's real bytes for the group (a batch's tables)."""
                adjust = getattr(self.memory, "adjust", None)
                if adjust is not None:
                    with self._cv:
                        adjust(handle, actual)
            try:
                self.executor(slot, group, report)
            except Exception as e:  # the loop keeps serving; the group fails
                for r in group:
                    r.error = f"{type(e).__name__}: {e}"
            t1 = time.perf_counter()
            with self._cv:
                for r in group:
                    r.t_done = t1
                    r.region = None
                    self.completed.append(r)
                    r.done.set()
                self.memory.release(handle)  # the executor has finished with the group's memory
                self._free_slots.append(slot)
                self._cv.notify_all()


class DevicePool:
    """The serving memory budget as one device buffer shared by every slot.
    A group reserves one contiguous region (first fit over the free list,
    offsets in 256-byte granules); release() returns it and merges it with
    free neighbours. Serving then allocates no device memory per request:
    allocating per request would go through the caching allocator, whose
    cached blocks belong to one stream each, and with several slots and very
    different sizes that churns device allocations and frees, which
    synchronize the device."""

    ALIGN = 256
    GROUP_MARGIN = 1 << 20       # reserved beyond a group's product bytes (batch tables, alignment)
    REQUEST_MARGIN = 64 << 10

    def margin(self, count: int) -> int:
        return self.GROUP_MARGIN + self.REQUEST_MARGIN * count

    def __init__(self, capacity: int, device):
        import torch
        self.capacity = (int(capacity) // self.ALIGN) * self.ALIGN
        self.buf = torch.empty(max(self.capacity, self.ALIGN), dtype=torch.uint8, device=device)
        self.free = [[0, self.capacity]]  # [offset, size], sorted by offset, never adjacent

    def largest_free(self) -> int:
        return max((n for _, n in self.free), default=0)

    def reserve(self, nbytes: int):
        n = (max(int(nbytes), 1) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for k, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    del self.free[k]
                else:
                    self.free[k] = [off + n, size - n]
                return Region(self, off, n)
        return None

    def release(self, region: "Region"):
        off, n = region.off, region.size
        k = 0
        while k < len(self.free) and self.free[k][0] < off:
            k += 1
        self.free.insert(k, [off, n])
        if k + 1 < len(self.free) and off + n == self.free[k + 1][0]:  # merge with the next block
            self.free[k][1] += self.free[k + 1][1]
            del self.free[k + 1]
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == off:  # and with the previous one
            self.free[k - 1][1] += self.free[k][1]
            del self.free[k]


class Region:
    """A group's reservation in a DevicePool: a bump allocator of 256-byte
    aligned pieces (uint8 device tensors). A request beyond the region (a
    batch's tables larger than the margin) gets its own block instead."""

    def __init__(self, pool: DevicePool, off: int, size: int):
        self.pool, self.off, self.size = pool, off, size
        self.used = 0
        self.overflow = 0

    def alloc(self, nbytes: int):
        import torch
        n = (max(int(nbytes), 1) + DevicePool.ALIGN - 1) // DevicePool.ALIGN * DevicePool.ALIGN
        if self.used + n > self.size:
            self.overflow += n
            return torch.empty(n, dtype=torch.uint8, device=self.pool.buf.device)
        t = self.pool.buf[self.off + self.used:self.off + self.used + n]
        self.used += n
        return t


class GpuExecutor:
    """Runs a group on the slot's own stream: one product as a plan, several
    as one batch, with workspaces (and the outputs of results that are not
    kept) carved from the slot's arena. Stores each request's DeviceCSR
    result (or its nnz when not kept) and reports the group's device bytes
    (workspaces and outputs) to the server."""

    def __init__(self, slots: int):
        import torch
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._sizes: Dict[Any, int] = {}

    def make_memory(self, capacity: int) -> DevicePool:
        """The server's budget as one device buffer (see DevicePool)."""
        return DevicePool(capacity, self.device)

    def bytes_of(self, operands, semiring: str) -> int:
        """product_bytes of a resident operand set, computed once."""
        return self.info_of(operands, semiring)[0]

    def info_of(self, operands, semiring: str):
        """(product_bytes, products) of a resident operand set, computed once."""
        key = (id(operands), semiring)
        if key not in self._sizes:
            A, B, M, comp = operands
            self._sizes[key] = product_info(A, B, M, comp, semiring)
        return self._sizes[key]

    def __call__(self, slot: int, group: List[Request], report: Optional[Callable[[int], None]] = None):
        import torch

        from . import Batch, Plan, out_dtype
        s = self.streams[slot]
        region = group[0].region
        alloc = region.alloc if isinstance(region, Region) else None
        with torch.cuda.stream(s):
            if len(group) == 1:
                r = group[0]
                A, B, M, comp = r.operands
                with Plan(A, B, M, complement=comp, semiring=r.semiring, alloc=alloc) as p:
                    C = p.execute(out_alloc=None if r.keep else alloc)
                    r.result = C if r.keep else int(C.colidx.numel())
            else:
                with Batch([r.operands for r in group], semiring=group[0].semiring, alloc=alloc) as b:
                    outs = b.bind_new_outputs(out_alloc=alloc, keep=[r.keep for r in group])
                    if report is not None:
                        width = out_dtype(group[0].semiring).itemsize
                        report(b.plan_workspace_bytes + b.workspace_bytes +
                               sum(rp.numel() * 8 + ci.numel() * (4 + width) for rp, ci, _ in outs))
                    b.execute()
                    for r, C in zip(group, b.results()):
                        r.result = C if r.keep else int(C.colidx.numel())
            s.synchronize()


def percentiles(values: List[float], qs=(50, 99)) -> Dict[str, float]:
    import numpy as np
    if not values:
        return {f"p{q}": float("nan") for q in qs}
    a = np.asarray(values)
    return {f"p{q}": float(np.percentile(a, q)) for q in qs}


def run_trace(server: Server, make_request: Callable[[int], Request], arrivals: List[float],
              timeout: float = 600.0) -> List[Request]:
    """Submits make_request(i) at the relative times `arrivals` (seconds) and
    waits for all of them."""
    server.start()
    reqs = []
    t0 = time.perf_counter()
    try:
        for i, at in enumerate(arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            r = make_request(i)
            r.t_arrival = t0 + at
            reqs.append(server.submit(r))
        deadline = time.perf_counter() + timeout
        for r in reqs:
            r.done.wait(timeout=max(0.0, deadline - time.perf_counter()))
    finally:
        server.stop()
    return reqs
