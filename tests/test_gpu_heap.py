"""GPU parity of the heap kind (Section "Masked Heap SpGEVM Algorithm"): a
k-way merge of the rows of B selected by a row of A, one lane per row, with
the mask applied before an iterator enters the heap.

Rows whose row of A has at most 8 entries run in the heap kernel; the tests
check that they do (bin counts) and compare every result with the oracle:
structure and integer values bit-exact. For FP64 the heap folds the products
of a column in the order of A's row, which is the order in which the oracle
adds them (its first product sets the value, each later one is added), so the
heap's FP64 values must equal the oracle's bit for bit as well."""
import zlib

import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import VKIND, assert_same, msp, torch_or_skip, up

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_pair_i64", "lor_land_bool", "plus_times_i32", "plus_times_i64"]
HEAP_CAP = 8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_or_skip()


def clip_rows(X, cap):
    """The first `cap` entries of every row of X."""
    keep = np.concatenate([np.arange(X.rowptr[i], min(X.rowptr[i + 1], X.rowptr[i] + cap))
                           for i in range(X.nrows)] + [np.zeros(0, np.int64)]).astype(np.int64)
    lens = np.minimum(np.diff(X.rowptr), cap)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return mspgen.CSR(X.nrows, X.ncols, rp, X.colidx[keep].copy(),
                      None if X.values is None else X.values[keep].copy())


def heap_problem(seed, m, k, n, da, db, dm, sr):
    A = clip_rows(mspgen.er(m, k, da, seed * 10 + 1, VKIND[sr]), HEAP_CAP)
    B = mspgen.er(k, n, db, seed * 10 + 2, VKIND[sr])
    M = mspgen.er(m, n, dm, seed * 10 + 3, None)
    return A, B, M


def run_plan(A, B, M, comp, sr, **kw):
    m = msp()
    with m.Plan(up(A, sr), up(B, sr), up(M), comp, sr, **kw) as p:
        C = p.execute()
        bins = dict(p.bin_units)
        bins["heap"] = bins["heap_lane"] + bins["heap_lane_long_mask"]  # both heap bins
        kinds = dict(p.kind_units)
    R = oracle.masked_spgemm(A, B, M, comp, sr)
    return C, R, bins, kinds


def check_exact(C, R, sr):
    assert_same(C, R, sr)
    if sr == "plus_times_f64":
        _, _, v = C.to_host()
        assert np.array_equal(v.view(np.uint64), R.values.view(np.uint64)), "fp64 fold order differs"


def rows_with_output_bound(A, B, M, comp):
    """Rows with at least one admitted product (min(admitted, products) > 0)."""
    deg_b = np.diff(B.rowptr)
    flops = np.array([deg_b[A.colidx[A.rowptr[i]:A.rowptr[i + 1]]].sum() for i in range(A.nrows)])
    mn = np.diff(M.rowptr)
    adm = (M.ncols - mn) if comp else mn
    return int(np.count_nonzero(np.minimum(adm, flops) > 0))


# narrow: dense state would fit one wave; wide: several 4096-column tiles; long: B rows longer than a wave
SHAPES = {"narrow": (300, 200, 400, 3.0, 6.0, 60.0), "wide": (257, 300, 9000, 4.0, 9.0, 300.0),
          "long": (200, 150, 5000, 2.5, 150.0, 900.0)}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("sr", SEMIRINGS)
@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("phase", [1, 2])
def test_forced_heap(shape, sr, comp, phase):
    A, B, M = heap_problem(zlib.crc32(f"{shape}/{sr}".encode()) % 1000 + 3, *SHAPES[shape], sr)
    C, R, bins, kinds = run_plan(A, B, M, comp, sr, force_kind="heap", phase=phase)
    check_exact(C, R, sr)
    units = rows_with_output_bound(A, B, M, comp)
    assert bins["heap"] == units and kinds["heap"] == units


def test_rows_too_long_for_the_heap_take_the_automatic_choice():
    sr = "plus_times_f64"
    A = mspgen.er(400, 300, 7.0, 71, "f64")  # some rows have more than 8 entries
    B = mspgen.er(300, 2000, 5.0, 72, "f64")
    M = mspgen.er(400, 2000, 100.0, 73, None)
    long_rows = int(np.count_nonzero(np.diff(A.rowptr) > HEAP_CAP))
    assert long_rows > 20
    for comp in (False, True):
        C, R, bins, _ = run_plan(A, B, M, comp, sr, force_kind="heap")
        assert_same(C, R, sr)
        assert 0 < bins["heap"] < rows_with_output_bound(A, B, M, comp)


def test_equal_columns_from_every_iterator():
    """Every row of B holds the same columns, so each output column gathers
    one product from every iterator of the heap (ties broken by slot)."""
    sr = "plus_times_f64"
    rng = np.random.default_rng(9)
    k, n = 50, 700
    cols = np.sort(rng.choice(n, size=40, replace=False))
    B = mspgen.from_coo(k, n, np.repeat(np.arange(k), len(cols)), np.tile(cols, k))
    B = B.with_values(rng.random(B.nnz))
    A = clip_rows(mspgen.er(120, k, 8.0, 74, "f64"), HEAP_CAP)
    M = mspgen.er(120, n, 200.0, 75, None)
    for comp in (False, True):
        for phase in (1, 2):
            C, R, bins, _ = run_plan(A, B, M, comp, sr, force_kind="heap", phase=phase)
            check_exact(C, R, sr)
            assert bins["heap"] == rows_with_output_bound(A, B, M, comp)


def test_explicit_zeros_and_wraparound_in_heap():
    rng = np.random.default_rng(4)
    A = clip_rows(mspgen.er(200, 150, 5, 81, "i32"), HEAP_CAP)
    B = mspgen.er(150, 300, 8, 82, "i32")
    A.values[rng.integers(0, A.nnz, 100)] = 0
    A.values[:] = A.values * 40000
    B.values[:] = B.values * 30000
    M = mspgen.er(200, 300, 60, 83, None)
    for comp in (False, True):
        C, R, _, _ = run_plan(A, B, M, comp, "plus_times_i32", force_kind="heap")
        check_exact(C, R, "plus_times_i32")
    Ab = clip_rows(mspgen.er(200, 150, 5, 84, "u8"), HEAP_CAP)
    Ab.values[::2] = 0  # stored false entries still give structural products
    Bb = mspgen.er(150, 300, 8, 85, "u8")
    C, R, _, _ = run_plan(Ab, Bb, M, False, "lor_land_bool", force_kind="heap")
    check_exact(C, R, "lor_land_bool")


def test_auto_picks_heap_for_light_rows():
    """Very sparse A and B against a denser mask (the regime the paper's
    heap targets): the automatic binner sends the light rows to the heap;
    heap_flops = 0 turns that off. Same result either way."""
    sr = "plus_times_f64"
    A = mspgen.er(3000, 3000, 1.5, 91, "f64")
    B = mspgen.er(3000, 3000, 1.5, 92, "f64")
    M = mspgen.er(3000, 3000, 64.0, 93, None)
    C, R, bins, _ = run_plan(A, B, M, False, sr)
    assert_same(C, R, sr)
    assert bins["heap"] > 1000
    C0, _, bins0, _ = run_plan(A, B, M, False, sr, heap_flops=0)
    assert_same(C0, R, sr)
    assert bins0["heap"] == 0
    # light rows under a complemented mask
    Mc = mspgen.er(3000, 3000, 10.0, 94, None)
    C, R, bins, _ = run_plan(A, B, Mc, True, sr)
    assert_same(C, R, sr)
    assert bins["heap"] > 1000
    # a complemented mask wider than one 4096-column dense tile: rows of at most heap_flops
    # products take the heap, heavier ones are sorted; with a large heap_flops every fitting
    # row takes the heap, however many products it has
    A2 = clip_rows(mspgen.er(2000, 500, 4.0, 95, "f64"), HEAP_CAP)
    B2 = mspgen.er(500, 10000, 20.0, 96, "f64")
    M2 = mspgen.er(2000, 10000, 50.0, 97, None)
    deg_b = np.diff(B2.rowptr)
    flops = np.array([deg_b[A2.colidx[A2.rowptr[i]:A2.rowptr[i + 1]]].sum() for i in range(A2.nrows)])
    C, R, bins, _ = run_plan(A2, B2, M2, True, sr)
    assert_same(C, R, sr)
    assert bins["heap"] == int(((flops > 0) & (flops <= 32)).sum()) > 0
    assert bins["sort_block"] == int((flops > 32).sum()) > 0
    C, R, bins, _ = run_plan(A2, B2, M2, True, sr, heap_flops=1 << 20)
    assert_same(C, R, sr)
    assert bins["heap"] == rows_with_output_bound(A2, B2, M2, True)


@pytest.mark.parametrize("n,sr,dm", [(5000, "plus_times_f64", 24.0), (120000, "plus_times_f64", 24.0),
                                     (120000, "plus_times_i32", 24.0), (120000, "lor_land_bool", 24.0),
                                     (5000, "plus_times_f64", 400.0), (40000, "plus_times_i64", 400.0)])
def test_auto_heap_small_and_large_bins(n, sr, dm):
    """A small automatic heap bin (normal mask) runs inside the launch of its
    mask-indexed neighbour: the wave kernel for mask rows of at most 256
    entries (bins of at most 32768 units), the block kernel for longer ones
    (at most 4096 units); a larger one runs in the heap kernel. Both agree
    with the oracle in both phases."""
    A = mspgen.er(n, n, 1.2, 301, VKIND[sr])
    B = mspgen.er(n, n, 1.2, 302, VKIND[sr])
    M = mspgen.er(n, n, dm, 303, None)
    for phase in (1, 2):
        C, R, bins, _ = run_plan(A, B, M, False, sr, phase=phase)
        assert_same(C, R, sr)
        key = "heap_lane_long_mask" if dm > 256 else "heap_lane"
        assert bins[key] == bins["heap"] and (bins["heap"] > (4096 if dm > 256 else 32768)) == (n > 10000)


def test_triangle_counting_heap():
    L = mspgen.triangle_input(11, 16, 5)
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    for phase in (1, 2):
        C, _, bins, _ = run_plan(L, L, L, False, "plus_pair_i64", force_kind="heap", phase=phase)
        assert_same(C, R, "plus_pair_i64")
        assert bins["heap"] > 0


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_i32", "lor_land_bool"])
def test_heap_in_batch(sr):
    torch = torch_or_skip()
    m = msp()
    probs = []
    for t, (mm, k, n, da, db, dm, comp) in enumerate([(300, 200, 400, 3, 6, 60, False), (150, 300, 7000, 2, 9, 500, True),
                                                      (1, 5, 5, 2, 2, 2, False), (0, 10, 10, 1, 1, 1, False),
                                                      (400, 300, 3000, 6, 5, 40, False)]):
        A, B, M = heap_problem(40 + t, mm, k, n, da, db, dm, sr)
        probs.append((A, B, M, comp))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    with m.Batch(dev, semiring=sr, force_kind="heap") as b:
        b.bind_new_outputs()
        b.execute()
        assert b.bin_units["heap_lane"] + b.bin_units["heap_lane_long_mask"] > 0
        for (A, B, M, c), C, d in zip(probs, b.results(), dev):
            check_exact(C, oracle.masked_spgemm(A, B, M, c, sr), sr)
            single = m.masked_spgemm(d[0], d[1], d[2], complement=c, semiring=sr, force_kind="heap")
            assert torch.equal(single.rowptr, C.rowptr) and torch.equal(single.colidx, C.colidx)
            assert torch.equal(single.values, C.values)
