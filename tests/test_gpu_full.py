"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times: triangle counting on R-MAT scale 18 compared entry by entry
with the oracle; the 512-source BFS step on R-MAT scale 20, int32 on every
row and boolean on the whole row-pointer array plus sampled rows; the
64-product batch at full size on sampled rows of every product; light Erdos-Renyi products of the density heatmap that run in
the heap kind, in full."""
import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import assert_same, msp, torch_or_skip, up

pytestmark = pytest.mark.gpu


def test_triangle_counting_full_size():
    L = mspgen.triangle_input(18, 16, 18)
    dL = up(L)
    C = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64")
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    assert_same(C, R, "plus_pair_i64")
    assert int(msp().reduce(C.values, "plus_pair_i64").item()) == int(R.values.sum())


@pytest.fixture(scope="module")
def bfs_case():
    """R-MAT scale 20 graph, the 512-source frontiers with path counts, and
    the oracle's whole int32 result (every row)."""
    G = mspgen.rmat_graph(20, 16, 20)
    F, V, srcs, lv = mspgen.bfs_step_input(G, 512, 21, "i64")
    Fi = F.with_values(F.values.astype(np.int32))
    R = oracle.masked_spgemm(G, Fi, V, True, "plus_times_i32")
    return G, F, V, R


def test_bfs_step_full_size_int32_every_row(bfs_case):
    """The int32 path-count step compared with the oracle on every row:
    row pointers, column indices and values."""
    G, F, V, R = bfs_case
    sr = "plus_times_i32"
    C = msp().masked_spgemm(up(G), up(F.with_values(F.values.astype(np.int32)), sr), up(V), complement=True,
                            semiring=sr)
    assert_same(C, R, sr)


def test_bfs_step_full_size_bool(bfs_case):
    """The boolean step: the whole row-pointer array against the oracle's
    (an entry exists under either semiring exactly when some product is
    stored, so both patterns agree), and sampled rows (a uniform sample plus
    the 20 hubs) in full against the boolean oracle."""
    G, F, V, R = bfs_case
    sr = "lor_land_bool"
    Fb = F.with_values(np.ones(F.nnz, np.uint8))
    C = msp().masked_spgemm(up(G), up(Fb, sr), up(V), complement=True, semiring=sr)
    rp = C.rowptr.cpu().numpy()
    assert np.array_equal(rp, R.rowptr)
    rng = np.random.default_rng(5)
    deg = np.diff(G.rowptr)
    hubs = np.argsort(deg)[-20:]
    rows = np.unique(np.concatenate([rng.integers(0, G.nrows, 3000), hubs]))
    Rb = oracle.masked_spgemm(G, Fb, V, True, sr, rows=rows)
    assert_same(C, Rb, sr, rows=rows)


def test_batch_full_size_uncapped_sampled():
    """The 64-product FP64 batch at full size (masks uncapped: about 5.5e9
    mask entries in all), run as one batch replayed from a captured graph;
    sampled rows of every product (a uniform sample plus the product's
    heaviest rows by products and by mask length) against the oracle, whose
    mask rows are drawn one by one from the same per-row streams."""
    torch = torch_or_skip()
    m = msp()
    prms = mspgen.batch_params(64, seed=4)
    dev, host = [], []
    for prm in prms:
        A, B = mspgen.batch_operands(prm)
        M = mspgen.batch_mask(prm)
        dev.append((up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M), False))
        host.append((prm, A, B, np.diff(M.rowptr)))
        del M
    assert sum(int(h[3].sum()) for h in host) > 5_000_000_000
    rng = np.random.default_rng(9)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring="plus_times_f64") as b:
            b.bind_new_outputs()
            b.graph_launch()
            b.graph_launch()
            res = b.results()
    for (prm, A, B, mrow), C in zip(host, res):
        fl = np.bincount(np.repeat(np.arange(A.nrows), np.diff(A.rowptr)),
                         weights=np.diff(B.rowptr)[A.colidx], minlength=A.nrows)
        rows = np.unique(np.concatenate([rng.integers(0, A.nrows, 32), np.argsort(fl)[-4:], np.argsort(mrow)[-4:]]))
        Ms = mspgen.batch_mask_rows(prm, rows)
        R = oracle.masked_spgemm(A, B, Ms, False, "plus_times_f64", rows=rows)
        assert_same(C, R, "plus_times_f64", rows=rows)
        rp = C.rowptr.cpu().numpy()
        assert np.all(np.diff(rp) >= 0) and rp[-1] == C.colidx.numel()


@pytest.mark.parametrize("d,dm,comp", [(1.0, 64.0, False), (4.0, 1024.0, False), (2.0, 8.0, True)])
def test_light_er_heap_sizes_full(d, dm, comp):
    """The density-heatmap regime where the heap kind carries the rows (inputs
    much sparser than the mask; a complemented mask over 2^20 columns),
    compared in full with the oracle at the heatmap's size."""
    n = 1 << 20 if dm < 1000 else 1 << 18
    A = mspgen.er(n, n, d, 11 + n, "f64")
    B = mspgen.er(n, n, d, 12 + n, "f64")
    M = mspgen.er(n, n, dm, 13 + n, None)
    with msp().Plan(up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M), comp, "plus_times_f64") as p:
        C = p.execute()
        assert p.bin_units["heap_lane"] + p.bin_units["heap_lane_long_mask"] > 32768
    assert_same(C, oracle.masked_spgemm(A, B, M, comp, "plus_times_f64"), "plus_times_f64")
