"""GPU parity of the sorting bin: rows under a complemented mask of a matrix
wider than one 4096-column dense tile, with more products than the heap
takes automatically (heap_flops, 32 by default) and at most 4096, are
expanded, sorted by column, folded and filtered against the mask row
(automatic choice only). Each case checks the bin ran and compares with the
oracle: patterns and integer values bit-exact, FP64 within 1e-12 relative."""
import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import VKIND, assert_same, msp, torch_or_skip, up

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_pair_i64", "lor_land_bool", "plus_times_i32", "plus_times_i64"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_or_skip()


def _plan_check(A, B, M, sr, complement=True, phase=1, **kw):
    m = msp()
    with m.Plan(up(A, sr), up(B, sr), up(M), complement, sr, phase=phase, **kw) as p:
        C = p.execute()
        bins = dict(p.bin_units)
    assert_same(C, oracle.masked_spgemm(A, B, M, complement, sr), sr)
    return bins


def _limits_problem(sr, seed=5):
    """Rows on both sides of each limit of the sorting bin, n = 45000 (eleven
    4096-column tiles: rows of 1024 products or more are sorted only from ten
    tiles on, fewer stream the dense tiles). B row b
    < 6000 has b % 65 entries; rows 6000..6099 all hold the same 34 columns,
    0 and n - 1 among them. Row types (cycled): 9 entries of A with 256
    products (sorted); 8 entries of A with 160 products (sorted); 64 entries
    with 4096 products (sorted); 65 entries with 4097 products (dense tiles);
    40 entries of which most have empty B rows, under a mask row that holds
    all but five product columns (sorted); 20 entries whose 680 products
    fold into 34 columns (sorted); entries whose B rows are all empty (no
    products); 4 entries with 32 products (heap); 3 entries with 33 products
    (sorted)."""
    rng = np.random.default_rng(seed)
    n, k = 45000, 6100
    blen = np.arange(k) % 65
    bcols = [np.sort(rng.choice(n, size=blen[b], replace=False)) for b in range(k)]
    shared = np.sort(np.concatenate([[0, n - 1], rng.choice(np.arange(1, n - 1), size=32, replace=False)]))
    for b in range(6000, k):
        bcols[b] = shared
    B = mspgen.from_coo(k, n, np.concatenate([np.full(len(c), b) for b, c in enumerate(bcols)]),
                        np.concatenate(bcols))
    by_len = {L: np.nonzero(blen[:6000] == L)[0] for L in range(65)}
    pick = lambda L, c: rng.choice(by_len[L], size=c, replace=False)  # noqa: E731
    arows, acols, mrows, mcols = [], [], [], []
    m = 180
    for i in range(m):
        t = i % 9
        ent = [
            lambda: np.concatenate([pick(32, 8), pick(0, 1)]),
            lambda: pick(20, 8),
            lambda: pick(64, 64),
            lambda: np.concatenate([pick(64, 64), pick(1, 1)]),
            lambda: np.concatenate([pick(0, 36), pick(25, 4)]),
            lambda: 6000 + rng.choice(100, size=20, replace=False),
            lambda: pick(0, 12),
            lambda: pick(8, 4),
            lambda: np.concatenate([pick(11, 3)]),
        ][t]()
        ent = np.unique(ent.astype(np.int64))
        arows.append(np.full(len(ent), i))
        acols.append(ent)
        prod = np.unique(np.concatenate([bcols[b] for b in ent]))
        if t == 4:
            mc = prod[: len(prod) - 5]
        else:
            third = rng.choice(prod, size=len(prod) // 3, replace=False) if len(prod) else prod
            mc = np.unique(np.concatenate([third, rng.choice(n, size=50, replace=False)]))
        mrows.append(np.full(len(mc), i))
        mcols.append(mc)
    A = mspgen.from_coo(m, k, np.concatenate(arows), np.concatenate(acols))
    M = mspgen.from_coo(m, n, np.concatenate(mrows), np.concatenate(mcols))
    vk = VKIND[sr]
    A = A.with_values(mspgen.random_values(A.nnz, vk, np.random.default_rng(seed + 10)))
    B = B.with_values(mspgen.random_values(B.nnz, vk, np.random.default_rng(seed + 20)))
    return A, B, M


def _row_classes(A, B):
    alen = np.diff(A.rowptr)
    bl = np.diff(B.rowptr)
    fl = np.array([bl[A.colidx[A.rowptr[i]:A.rowptr[i + 1]]].sum() for i in range(A.nrows)])
    return alen, fl


@pytest.mark.parametrize("phase", [1, 2])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_sorting_limits(sr, phase):
    A, B, M = _limits_problem(sr)
    alen, fl = _row_classes(A, B)
    expect = int(((fl > 32) & (fl <= 4096)).sum())
    bins = _plan_check(A, B, M, sr, phase=phase)
    assert bins["sort_block"] == expect and expect > 0, (bins, expect)
    assert bins["heap_lane"] == int(((fl > 0) & (fl <= 32)).sum()) > 0
    assert bins["dense_block"] == int((fl > 4096).sum()) * 11  # 45000 columns: eleven 4096-column tiles


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_i32"])
def test_forced_dense_never_sorts(sr):
    A, B, M = _limits_problem(sr, seed=6)
    bins = _plan_check(A, B, M, sr, force_kind="dense")
    assert bins["sort_block"] == 0


def test_normal_mask_never_sorts():
    A, B, M = _limits_problem("plus_times_f64", seed=7)
    bins = _plan_check(A, B, M, "plus_times_f64", complement=False)
    assert bins["sort_block"] == 0


def test_wide_complement_heavy_rows():
    """2000 rows of about 16 entries over a graph of 2^20 vertices under a
    complemented mask of degree 8: every row with more than 32 products
    sorts (the tiled dense kind would restream each such row 256 times)."""
    n = 1 << 20
    A = mspgen.er(2000, n, 16.0, 41, "f64")
    B = mspgen.er(n, n, 16.0, 42, "f64")
    M = mspgen.er(2000, n, 8.0, 43, None)
    m = msp()
    dA, dB, dM = up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M)
    with m.Plan(dA, dB, dM, True, "plus_times_f64") as p:
        C = p.execute()
        _, fl = _row_classes(A, B)
        assert p.bin_units["sort_block"] == int((fl > 32).sum()) > 1900
    assert_same(C, oracle.masked_spgemm(A, B, M, True, "plus_times_f64"), "plus_times_f64")


@pytest.mark.parametrize("sr", ["plus_times_f64", "lor_land_bool"])
def test_sorting_rows_in_a_batch(sr):
    torch = torch_or_skip()
    m = msp()
    probs = [(*_limits_problem(sr, seed=8), True), (*_limits_problem(sr, seed=9), True)]
    n = 1 << 16
    probs.append((mspgen.er(500, n, 12.0, 51, VKIND[sr]), mspgen.er(n, n, 12.0, 52, VKIND[sr]),
                  mspgen.er(500, n, 8.0, 53, None), True))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            assert b.bin_units["sort_block"] > 0
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
                for (A, B, M, c), C in zip(probs, b.results()):
                    assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_i32"])
def test_small_heap_bin_of_mixed_masks_runs_sorted(sr):
    """A batch whose light rows (heap bin) come from products with normal and
    with complemented masks: no mask-indexed launch can take the complemented
    ones, so the small bin runs in the one-wave sorting kernel, which filters
    each row by its own product's mask mode."""
    torch = torch_or_skip()
    m = msp()
    probs = []
    for t, (rows, n, d, dm, comp) in enumerate([(3000, 3000, 1.5, 64.0, False), (2000, 9000, 1.5, 10.0, True),
                                               (1500, 1500, 2.0, 30.0, False), (1200, 70000, 1.2, 6.0, True)]):
        A = mspgen.er(rows, n, d, 600 + 3 * t, VKIND[sr])
        B = mspgen.er(n, n, d, 601 + 3 * t, VKIND[sr])
        M = mspgen.er(rows, n, dm, 602 + 3 * t, None)
        probs.append((A, B, M, comp))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            assert 0 < b.bin_units["heap_lane"] <= 32768
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
                for (A, B, M, c), C in zip(probs, b.results()):
                    assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)


def _wide_problem(sr):
    """300 rows over 2^25 columns: even rows about 150 products, odd rows
    about 750; B holds columns 2^24 - 1, 2^24 and n - 1 among others."""
    rng = np.random.default_rng(70)
    n, k, m = 1 << 25, 3000, 300
    B = mspgen.er(k, n, 24.0, 71, VKIND[sr])
    extra = np.array([(1 << 24) - 1, 1 << 24, n - 1], np.int64)
    rows = np.concatenate([np.repeat(np.arange(B.nrows), np.diff(B.rowptr)), rng.integers(0, k, size=60)])
    cols = np.concatenate([B.colidx.astype(np.int64), rng.choice(extra, size=60)])
    B = mspgen.from_coo(k, n, rows, cols)
    B = B.with_values(mspgen.random_values(B.nnz, VKIND[sr], np.random.default_rng(72)))
    alen = np.where(np.arange(m) % 2 == 0, 6, 30)
    A = mspgen.from_coo(m, k, np.repeat(np.arange(m), alen),
                        np.concatenate([np.sort(rng.choice(k, size=a, replace=False)) for a in alen]))
    A = A.with_values(mspgen.random_values(A.nnz, VKIND[sr], np.random.default_rng(73)))
    M = mspgen.er(m, n, 5.0, 74, None)
    return A, B, M


@pytest.mark.parametrize("sr,phase", [("plus_times_f64", 1), ("plus_pair_i64", 1), ("plus_times_i32", 2),
                                      ("lor_land_bool", 2)])
def test_columns_beyond_32_bit_keys(sr, phase):
    """Over 2^25 columns the one-wave sorting kernels keep 64-bit keys (below
    2^22 columns, or 2^24 for rows under 256 products, a key fits 32 bits).
    The oracle runs on one thread (its accumulator spans all n columns)."""
    A, B, M = _wide_problem(sr)
    mm = msp()
    with mm.Plan(up(A, sr), up(B, sr), up(M), True, sr, phase=phase) as p:
        assert p.bin_units["sort_block"] == A.nrows
        C = p.execute()
    assert_same(C, oracle.masked_spgemm(A, B, M, True, sr, nthreads=1), sr)


def test_key_width_of_a_batch_follows_its_widest_product():
    """A batch holding a 2^16-column product and the 2^25-column one sorts
    both with 64-bit keys (the width is chosen per launch)."""
    torch = torch_or_skip()
    sr = "plus_times_f64"
    m = msp()
    n = 1 << 16
    probs = [(mspgen.er(800, n, 16.0, 91, VKIND[sr]), mspgen.er(n, n, 16.0, 92, VKIND[sr]),
              mspgen.er(800, n, 8.0, 93, None), True), (*_wide_problem(sr), True)]
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    with m.Batch(dev, semiring=sr) as b:
        assert b.bin_units["sort_block"] > 1000
        b.bind_new_outputs()
        b.execute()
        for (A, B, M, c), C in zip(probs, b.results()):
            assert_same(C, oracle.masked_spgemm(A, B, M, c, sr, nthreads=1), sr)


@pytest.mark.parametrize("n", [8192, 40960])
def test_heavy_rows_sort_only_over_many_tiles(n):
    """Rows of 1024 to 4096 products under a complemented mask: over 2 tiles
    they stream the dense tiles, over 10 tiles they are sorted."""
    sr = "plus_times_f64"
    A = mspgen.er(400, n, 40.0, 81, VKIND[sr])
    B = mspgen.er(n, n, 40.0, 82, VKIND[sr])
    M = mspgen.er(400, n, 30.0, 83, None)
    _, fl = _row_classes(A, B)
    heavy = int(((fl >= 1024) & (fl <= 4096)).sum())
    assert heavy > 300
    bins = _plan_check(A, B, M, sr)
    if n == 8192:
        assert bins["sort_block"] == int(((fl > 32) & (fl < 1024)).sum())
        assert bins["dense_block"] == 2 * int((fl >= 1024).sum())
    else:
        assert bins["sort_block"] == int(((fl > 32) & (fl <= 4096)).sum())
