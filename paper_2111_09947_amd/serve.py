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
  - Admission is by memory: a request's device bytes must fit the budget
    minus what running groups hold; otherwise it waits. The bytes are the
    library's own sizes for the product (plan workspace, execution workspace
    and the output at its upper bound: product_bytes), taken once per
    resident operand set. A batch's device tables add a little to the sum of
    its products; the executor reports the group's real bytes and the
    accounting follows them while the group runs. A request that alone
    exceeds the budget, or whose execution raises, completes with an error
    and the loop keeps serving.
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
    t_arrival: float = 0.0      # perf_counter() time of arrival
    t_start: float = 0.0
    t_done: float = 0.0
    result: Any = None
    keep: bool = False          # keep the result (otherwise dropped after completion)
    error: Optional[str] = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def product_bytes(A, B, M, complement: bool, semiring: str) -> int:
    """Device bytes one product takes in the library: its plan workspace,
    its execution workspace and its output (row pointers, and column indices
    and values at the upper bound), as the library's size queries give them.
    Runs the row analysis once (one plan creation)."""
    from . import Plan, out_dtype
    with Plan(A, B, M, complement=complement, semiring=semiring) as p:
        width = out_dtype(semiring).itemsize
        return (p.plan_workspace_bytes + p.workspace_bytes + 8 * (p.nrows + 1)
                + max(p.upper_bound, 1) * (4 + width))


class Server:
    def __init__(self, executor: Callable[[int, List[Request]], None], slots: int = 4, max_batch: int = 8,
                 mem_budget: int = 64 << 30, continuous: bool = True):
        self.executor = executor
        self.slots = slots if continuous else 1
        self.max_batch = max_batch if continuous else 1
        self.mem_budget = mem_budget
        self.continuous = continuous
        self._queue: Deque[Request] = collections.deque()
        self._cv = threading.Condition()
        self._free_slots = list(range(self.slots))
        self._mem_in_use = 0
        self._running = False
        self._threads: List[threading.Thread] = []
        self._work: Dict[int, Deque[List[Request]]] = {s: collections.deque() for s in range(self.slots)}
        self.completed: List[Request] = []

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
        that fit the remaining memory budget."""
        head = self._queue[0]
        room = self.mem_budget - self._mem_in_use
        if head.mem_bytes > self.mem_budget:
            self._queue.popleft()
            head.error = "request exceeds the memory budget"
            head.t_done = time.perf_counter()
            head.done.set()
            self.completed.append(head)
            return []
        if head.mem_bytes > room:
            return []  # wait for memory
        group = [self._queue.popleft()]
        room -= head.mem_bytes
        if self.continuous:
            keep: Deque[Request] = collections.deque()
            while self._queue and len(group) < self.max_batch:
                r = self._queue.popleft()
                if r.semiring == head.semiring and r.mem_bytes <= room:
                    group.append(r)
                    room -= r.mem_bytes
                else:
                    keep.append(r)
            keep.extend(self._queue)
            self._queue = keep
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
                    if self._queue and self._queue[0].mem_bytes <= self.mem_budget:
                        self._cv.wait(timeout=0.01)  # memory is held by running groups
                    continue
                slot = self._free_slots.pop(0)
                self._mem_in_use += sum(r.mem_bytes for r in group)
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
            admitted = sum(r.mem_bytes for r in group)
            held = admitted

            def report(actual: int):
                """The executor's real bytes for the group (a batch's tables)."""
                nonlocal held
                with self._cv:
                    self._mem_in_use += int(actual) - held
                    held = int(actual)
            try:
                self.executor(slot, group, report)
            except Exception as e:  # the loop keeps serving; the group fails
                for r in group:
                    r.error = f"{type(e).__name__}: {e}"
            t1 = time.perf_counter()
            with self._cv:
                for r in group:
                    r.t_done = t1
                    self.completed.append(r)
                    r.done.set()
                self._mem_in_use -= held
                self._free_slots.append(slot)
                self._cv.notify_all()


class GpuExecutor:
    """Runs a group on the slot's own stream: one product as a plan, several
    as one batch. Stores each request's DeviceCSR result and reports the
    group's device bytes (workspaces and outputs) to the server."""

    def __init__(self, slots: int):
        import torch
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self._sizes: Dict[Any, int] = {}

    def bytes_of(self, operands, semiring: str) -> int:
        """product_bytes of a resident operand set, computed once."""
        key = (id(operands), semiring)
        if key not in self._sizes:
            A, B, M, comp = operands
            self._sizes[key] = product_bytes(A, B, M, comp, semiring)
        return self._sizes[key]

    def __call__(self, slot: int, group: List[Request], report: Optional[Callable[[int], None]] = None):
        import torch

        from . import Batch, Plan, out_dtype
        s = self.streams[slot]
        with torch.cuda.stream(s):
            if len(group) == 1:
                r = group[0]
                A, B, M, comp = r.operands
                with Plan(A, B, M, complement=comp, semiring=r.semiring) as p:
                    C = p.execute()
                    r.result = C if r.keep else int(C.colidx.numel())
            else:
                with Batch([r.operands for r in group], semiring=group[0].semiring) as b:
                    outs = b.bind_new_outputs()
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
