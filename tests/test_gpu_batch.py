"""GPU parity of batches: every product of a batch (one launch per kernel bin
for all products, optionally replayed from a captured HIP graph) equals the
oracle and the same product run alone."""
import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import assert_same, msp, torch_or_skip, up

pytestmark = pytest.mark.gpu


def _mixed_problems(seed, sr="plus_times_f64"):
    vk = {"plus_times_f64": "f64", "plus_pair_i64": "f64", "plus_times_i32": "i32", "lor_land_bool": "u8"}[sr]
    rng = np.random.default_rng(seed)
    probs = []
    shapes = [(300, 200, 400, 5, 6, 30, False), (150, 700, 9000, 9, 7, 80, False), (1, 5, 5, 2, 2, 2, False),
              (0, 10, 10, 1, 1, 1, False), (400, 300, 500, 4, 5, 50, True), (200, 100, 20000, 30, 40, 3000, False),
              (64, 64, 64, 8, 8, 8, True), (100, 50, 3000, 20, 100, 10, False)]
    for t, (m, k, n, da, db, dm, comp) in enumerate(shapes):
        s = int(rng.integers(1, 10**6))
        A = mspgen.er(m, k, da, s + 1, vk)
        B = mspgen.er(k, n, db, s + 2, vk)
        M = mspgen.er(m, n, dm, s + 3, None)
        probs.append((A, B, M, comp))
    return probs


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_pair_i64", "plus_times_i32", "lor_land_bool"])
def test_batch_matches_oracle_and_single(sr):
    torch = torch_or_skip()
    m = msp()
    probs = _mixed_problems(7, sr)
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    with m.Batch(dev, semiring=sr) as b:
        # the mix has light rows that the binner merges in the heap kind (small bins run inside
        # the mask-indexed launches of the batch)
        assert b.bin_units["heap_lane"] + b.bin_units["heap_lane_long_mask"] > 0
        b.bind_new_outputs()
        b.execute()
        res = b.results()
        for (A, B, M, c), C, d in zip(probs, res, dev):
            R = oracle.masked_spgemm(A, B, M, c, sr)
            assert_same(C, R, sr)
            single = m.masked_spgemm(d[0], d[1], d[2], complement=c, semiring=sr)
            assert torch.equal(single.rowptr, C.rowptr) and torch.equal(single.colidx, C.colidx)
            if sr != "plus_times_f64":
                assert torch.equal(single.values, C.values)


def test_batch_graph_replays():
    """The captured graph replayed several times, with unrelated eager work
    and synchronizations in between, gives the oracle's result every time."""
    torch = torch_or_skip()
    m = msp()
    sr = "plus_times_f64"
    probs = _mixed_problems(11, sr)
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    refs = [oracle.masked_spgemm(A, B, M, c, sr) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            outs = b.bind_new_outputs()
            for rep in range(4):
                for (rp, ci, v) in outs:  # poison the outputs between replays
                    rp.fill_(-1)
                    ci.fill_(-1)
                    v.fill_(float("nan"))
                b.graph_launch()
                x = torch.ones(1 << 20, device="cuda") * rep  # eager work on the same stream
                s.synchronize()
                assert float(x.sum().item()) == float(rep * (1 << 20))
                for C, R in zip(b.results(), refs):
                    assert_same(C, R, sr)


def test_batch_rebind_changes_outputs():
    torch = torch_or_skip()
    m = msp()
    sr = "plus_pair_i64"
    probs = _mixed_problems(13, sr)
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            b.bind_new_outputs()
            b.graph_launch()
            first = [(C.colidx.clone(), C.values.clone()) for C in b.results()]
            b.bind_new_outputs()
            b.graph_launch()
            for (ci, v), C in zip(first, b.results()):
                assert torch.equal(ci, C.colidx) and torch.equal(v, C.values)


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_pair_i64"])
def test_batch_with_pull_costs_plans_product_by_product(sr):
    """With inner_ratio > 0 (pull costs per row, B^T built by the plan) the
    batch plan analyses its products one launch each; the results must be
    the oracle's either way, and the same as with the one-launch analysis."""
    torch = torch_or_skip()
    m = msp()
    probs = _mixed_problems(17, sr)
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    with m.Batch(dev, semiring=sr, inner_ratio=4) as b:
        b.bind_new_outputs()
        b.execute()
        pulled = b.results()
    with m.Batch(dev, semiring=sr) as b:
        b.bind_new_outputs()
        b.execute()
        pushed = b.results()
    for (A, B, M, c), C, D in zip(probs, pulled, pushed):
        R = oracle.masked_spgemm(A, B, M, c, sr)
        assert_same(C, R, sr)
        assert_same(D, R, sr)
        assert torch.equal(C.rowptr, D.rowptr) and torch.equal(C.colidx, D.colidx)


def test_batch_with_long_b_and_empty_products():
    """One-launch batch analysis over products of very different shapes: a B
    with more than 2^18 rows (its row lengths come from the 2-byte copy), a
    product with no rows, one with no entries in A, and ordinary ones."""
    torch = torch_or_skip()
    m = msp()
    sr = "plus_times_i32"
    rng = np.random.default_rng(23)
    probs = []
    kbig = (1 << 18) + 1000
    A = mspgen.er(500, kbig, 40.0, 31, "i32")
    B = mspgen.er(kbig, 3000, 3.0, 32, "i32")
    M = mspgen.er(500, 3000, 60.0, 33, None)
    probs.append((A, B, M, False))
    probs.append((mspgen.er(0, 10, 1.0, 34, "i32"), mspgen.er(10, 10, 1.0, 35, "i32"), mspgen.er(0, 10, 1.0, 36, None),
                  False))
    probs.append((mspgen.er(50, 40, 0.0, 37, "i32"), mspgen.er(40, 700, 5.0, 38, "i32"),
                  mspgen.er(50, 700, 9.0, 39, None), False))
    for t in range(3):
        s = int(rng.integers(1, 10**6))
        probs.append((mspgen.er(2000, 2000, 6.0, s, "i32"), mspgen.er(2000, 2000, 6.0, s + 1, "i32"),
                      mspgen.er(2000, 2000, 6.0, s + 2, None), t == 2))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
                for (A, B, M, c), C in zip(probs, b.results()):
                    assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)
