"""Serving on the GPU: a short Poisson trace through the continuous-batching
server (slots on their own streams, same-semiring groups run as one batch,
admission by the library's device bytes). Every request's result is
compared with the oracle (in full for small items, on sampled rows for the
large ones) and with the same product run alone: bit-exact for the integer
semiring, within 1e-12 relative for FP64. A second trace with a memory
budget that holds one large request at a time shows requests deferred for
memory and then served."""
import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import assert_same, msp, torch_or_skip

pytestmark = pytest.mark.gpu


def _pool():
    """(name, host operands (A, B, M, complement), semirings, rows to check or None = all)."""
    items = []
    for s in range(3):
        A = mspgen.er(4096, 4096, 8.0, 101 + 10 * s, "f64")
        B = mspgen.er(4096, 4096, 8.0, 102 + 10 * s, "f64")
        M = mspgen.er(4096, 4096, 8.0, 103 + 10 * s, None)
        items.append(("er4096", (A, B, M, False), ("plus_pair_i64", "plus_times_f64"), None))
    L = mspgen.triangle_input(16, 16, 18)
    items.append(("tc_rmat16", (L, L, L, False), ("plus_pair_i64",), None))
    G = mspgen.rmat_graph(16, 16, 20)
    F, V, _, _ = mspgen.bfs_step_input(G, 512, 21, "i64")
    items.append(("bfs_rmat16", (G.with_values(np.ones(G.nnz)), F.with_values(F.values.astype(np.float64)), V,
                                 True), ("plus_pair_i64", "plus_times_f64"), None))
    rng = np.random.default_rng(3)
    for prm in mspgen.batch_params(64, seed=4)[:12]:
        if prm["n"] * prm["md"] > 4e8:
            continue  # the heaviest masks are covered by the full-size batch test
        A, B = mspgen.batch_operands(prm)
        M = mspgen.batch_mask(prm)
        rows = np.unique(rng.integers(0, A.nrows, 48))
        items.append((f"mix{prm['t']}", (A, B, M, False), ("plus_pair_i64", "plus_times_f64"), rows))
    return items


@pytest.fixture(scope="module")
def pool():
    torch = torch_or_skip()
    m = msp()
    dev = torch.device("cuda:0")
    out = []
    for name, (A, B, M, c), srs, rows in _pool():
        d = (m.DeviceCSR.from_host(A, dev, torch.float64), m.DeviceCSR.from_host(B, dev, torch.float64),
             m.DeviceCSR.from_host(M, dev), c)
        out.append(dict(name=name, host=(A, B, M, c), dev=d, srs=srs, rows=rows))
    return out


def _check(item, sr, C, alone):
    """C (the served result) against the oracle and against the alone run."""
    torch = torch_or_skip()
    A, B, M, c = item["host"]
    rows = item["rows"]
    R = oracle.masked_spgemm(A, B, M, c, sr, rows=rows)
    assert_same(C, R, sr, rows=rows)
    assert torch.equal(C.rowptr, alone.rowptr) and torch.equal(C.colidx, alone.colidx)
    if sr == "plus_times_f64":
        assert bool(((C.values - alone.values).abs() <= 1e-12 * alone.values.abs()).all())
    else:
        assert torch.equal(C.values, alone.values)


def test_poisson_trace_matches_oracle_and_alone_runs(pool):
    m = msp()
    from paper_2111_09947_amd import serve
    rng = np.random.default_rng(17)
    seq = []
    for x in range(80):
        k = int(rng.integers(0, len(pool)))
        srs = pool[k]["srs"]
        seq.append((k, srs[int(rng.integers(0, len(srs)))]))
    ex = serve.GpuExecutor(3)
    sizes = {}

    def mk(i):
        k, sr = seq[i]
        key = (k, sr)
        if key not in sizes:
            sizes[key] = ex.bytes_of(pool[k]["dev"], sr)
        return serve.Request(rid=i, semiring=sr, operands=pool[k]["dev"], mem_bytes=sizes[key], keep=True)

    for i in range(len(seq)):  # sizes first, outside the timed trace
        mk(i)
    arrivals = list(np.cumsum(rng.exponential(0.002, size=len(seq))))
    srv = serve.Server(ex, slots=3, max_batch=6, mem_budget=32 << 30)
    reqs = serve.run_trace(srv, mk, arrivals, timeout=300)
    assert all(r.done.is_set() and r.error is None for r in reqs), [r.error for r in reqs if r.error]
    assert any(len(g) > 1 for g in _groups(reqs)), "no request was batched with another"
    alone = {}
    for r in reqs:
        k, sr = seq[r.rid]
        if (k, sr) not in alone:
            A, B, M, c = pool[k]["dev"]
            alone[(k, sr)] = m.masked_spgemm(A, B, M, complement=c, semiring=sr)
        _check(pool[k], sr, r.result, alone[(k, sr)])


def _groups(reqs):
    """Requests that started together (one group runs as one batch)."""
    by = {}
    for r in reqs:
        by.setdefault(r.t_start, []).append(r.rid)
    return list(by.values())


def test_memory_budget_defers_then_serves(pool):
    """A budget that holds one of the large requests at a time: all of them
    are served, correctly, one after another."""
    from paper_2111_09947_amd import serve
    big = max(range(len(pool)), key=lambda k: pool[k]["host"][2].nnz)
    sr = "plus_pair_i64"
    ex = serve.GpuExecutor(4)
    need = ex.bytes_of(pool[big]["dev"], sr)
    srv = serve.Server(ex, slots=4, max_batch=4, mem_budget=int(need * 1.5))
    reqs = serve.run_trace(srv, lambda i: serve.Request(rid=i, semiring=sr, operands=pool[big]["dev"],
                                                        mem_bytes=need, keep=True), [0.0] * 5, timeout=300)
    assert all(r.error is None for r in reqs), [r.error for r in reqs]
    spans = sorted((r.t_start, r.t_done) for r in reqs)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0 - 1e-6, "two requests that do not fit the budget together overlapped"
    m = msp()
    A, B, M, c = pool[big]["dev"]
    alone = m.masked_spgemm(A, B, M, complement=c, semiring=sr)
    for r in reqs:
        _check(pool[big], sr, r.result, alone)
    # a request larger than the whole budget completes with an error, and the loop keeps serving
    srv = serve.Server(ex, slots=2, max_batch=2, mem_budget=need // 2)
    r = serve.run_trace(srv, lambda i: serve.Request(rid=i, semiring=sr, operands=pool[big]["dev"], mem_bytes=need),
                        [0.0], timeout=60)[0]
    assert r.error and "budget" in r.error
