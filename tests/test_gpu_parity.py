"""GPU parity: the HIP path through the C-ABI against the CPU oracle.
rowptr/colidx bit-exact; integer values bit-exact; FP64 within 1e-12 relative."""
import math
import zlib

import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import (VKIND, assert_same, msp, rand_problem, run_and_check, torch_or_skip, up)

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_pair_i64", "lor_land_bool", "plus_times_i32", "plus_times_i64"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_or_skip()


# n = 400 fits the one-wave dense tile; n = 9000 needs three ragged 4096-column tiles
SHAPES = {"narrow": (300, 200, 400, 5.0, 6.0, 30.0), "wide": (257, 300, 9000, 7.0, 9.0, 60.0)}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("sr", SEMIRINGS)
@pytest.mark.parametrize("kind", ["auto", "dense", "hash", "maskidx", "inner"])
@pytest.mark.parametrize("phase", [1, 2])
def test_forced_kinds_normal_mask(shape, sr, kind, phase):
    A, B, M = rand_problem(zlib.crc32(f"{shape}/{sr}".encode()) % 1000, *SHAPES[shape], sr)
    run_and_check(A, B, M, False, sr, force_kind=kind, phase=phase)


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("sr", SEMIRINGS)
@pytest.mark.parametrize("phase", [1, 2])
def test_complemented_mask(shape, sr, phase):
    A, B, M = rand_problem(7 + len(shape), *SHAPES[shape], sr)
    run_and_check(A, B, M, True, sr, phase=phase)


@pytest.mark.parametrize("kind", ["auto", "hash", "maskidx", "dense", "inner"])
def test_heavy_rows_span_several_tiles(kind):
    """Mask rows longer than every LDS capacity (2048 mask entries per search
    tile, 512 hash entries, 4096-column tiles), A rows longer than one 64-entry batch and
    B rows longer than a wave."""
    rng = np.random.default_rng(5)
    m, k, n = 40, 300, 20000
    A = mspgen.er(m, k, 150.0, 11, "f64")
    B = mspgen.er(k, n, 120.0, 12, "f64")
    # mask rows of very different lengths: 0, tiny, ~1500, ~5000, ~12000
    dens = rng.choice([0.0, 3.0, 1500.0, 5000.0, 12000.0], size=m)
    rows, cols = [], []
    for i, d in enumerate(dens):
        c = np.unique(rng.integers(0, n, size=int(d)))
        rows.append(np.full(len(c), i))
        cols.append(c)
    M = mspgen.from_coo(m, n, np.concatenate(rows), np.concatenate(cols))
    run_and_check(A, B, M, False, "plus_times_f64", force_kind=kind)
    run_and_check(A, B, M, False, "plus_pair_i64", force_kind=kind, phase=2)


def test_complement_heavy_wide():
    A = mspgen.er(50, 80, 30.0, 21, "i32")
    B = mspgen.er(80, 10000, 200.0, 22, "i32")
    M = mspgen.er(50, 10000, 3000.0, 23, None)
    run_and_check(A, B, M, True, "plus_times_i32")
    run_and_check(A, B, M, True, "lor_land_bool", phase=2)


def test_more_units_than_one_dispatch_holds():
    """A complemented mask over 2^20 columns in the dense kind cuts every row
    into 256 column tiles, one 256-lane workgroup each: ~22M units, more
    than 2^32 work-items, so the bin runs as several launches over slices of
    its unit list (a single dispatch would silently leave units out)."""
    A = mspgen.er(120000, 120000, 2.0, 201, "i32")
    B = mspgen.er(120000, 1 << 20, 1.0, 202, "i32")
    M = mspgen.er(120000, 1 << 20, 4.0, 203, None)
    R = oracle.masked_spgemm(A, B, M, True, "plus_times_i32")
    for phase in (1, 2):
        with msp().Plan(up(A, "plus_times_i32"), up(B, "plus_times_i32"), up(M), True, "plus_times_i32",
                        phase=phase, force_kind="dense") as p:
            assert p.bin_units["dense_block"] * 256 > 1 << 32
            C = p.execute()
        assert_same(C, R, "plus_times_i32")


def _empty(m, n):
    return mspgen.CSR(m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32))


def _full(m, n):
    r, c = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    return mspgen.from_coo(m, n, r.ravel(), c.ravel())


@pytest.mark.parametrize("case", ["m0", "n0", "k0", "emptyA", "emptyM", "fullM", "onecol", "rect"])
@pytest.mark.parametrize("complement", [False, True])
def test_edge_shapes(case, complement):
    sr = "plus_times_f64"
    if case == "m0":
        A, B, M = mspgen.er(0, 30, 3, 1, "f64"), mspgen.er(30, 40, 3, 2, "f64"), _empty(0, 40)
    elif case == "n0":
        A, B, M = mspgen.er(30, 20, 3, 1, "f64"), mspgen.er(20, 0, 3, 2, "f64"), _empty(30, 0)
    elif case == "k0":
        A, B, M = mspgen.er(30, 0, 3, 1, "f64"), mspgen.er(0, 40, 3, 2, "f64"), mspgen.er(30, 40, 5, 3, None)
    elif case == "emptyA":
        A, B, M = _empty(30, 20), mspgen.er(20, 40, 3, 2, "f64"), mspgen.er(30, 40, 5, 3, None)
        A = A.with_values(np.zeros(0))
    elif case == "emptyM":
        A, B, M = mspgen.er(30, 20, 3, 1, "f64"), mspgen.er(20, 40, 3, 2, "f64"), _empty(30, 40)
    elif case == "fullM":
        A, B, M = mspgen.er(30, 20, 3, 1, "f64"), mspgen.er(20, 600, 30, 2, "f64"), _full(30, 600)
    elif case == "onecol":
        A, B, M = mspgen.er(64, 50, 4, 1, "f64"), mspgen.er(50, 1, 0.5, 2, "f64"), mspgen.er(64, 1, 0.6, 3, None)
    else:
        A, B, M = mspgen.er(7, 1000, 40, 1, "f64"), mspgen.er(1000, 3, 1.5, 2, "f64"), mspgen.er(7, 3, 2, 3, None)
    for phase in (1, 2):
        run_and_check(A, B, M, complement, sr, phase=phase)


def test_explicit_zeros_and_wraparound():
    rng = np.random.default_rng(3)
    A = mspgen.er(200, 150, 8, 31, "i32")
    B = mspgen.er(150, 300, 8, 32, "i32")
    A.values[rng.integers(0, A.nnz, 200)] = 0
    A.values[:] = A.values * 40000  # products exceed 2^31 and wrap
    B.values[:] = B.values * 30000
    M = mspgen.er(200, 300, 40, 33, None)
    for kind in ("auto", "dense", "hash", "maskidx", "inner"):
        run_and_check(A, B, M, False, "plus_times_i32", force_kind=kind)
    Af = mspgen.er(200, 150, 8, 34, "f64")
    Af.values[::3] = 0.0
    Bf = mspgen.er(150, 300, 8, 35, "f64")
    run_and_check(Af, Bf, M, False, "plus_times_f64")
    run_and_check(Af, Bf, M, True, "plus_times_f64")


def test_iso_valued_operands():
    A = mspgen.er(100, 90, 6, 41, None)
    B = mspgen.er(90, 120, 6, 42, None)
    M = mspgen.er(100, 120, 25, 43, None)
    for sr in SEMIRINGS:
        run_and_check(A, B, M, False, sr)


@pytest.mark.parametrize("n", [3, 8, 40, 100])
def test_complete_graph_triangles(n):
    L = mspgen.tril_strict(mspgen.complete_graph(n))
    dL = up(L)
    C = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64")
    rp, ci, v = C.to_host()
    assert int(rp[-1]) == math.comb(n - 1, 2)
    assert int(v.sum()) == math.comb(n, 3)
    s = msp().reduce(C.values, "plus_pair_i64")
    assert int(s.item()) == math.comb(n, 3)


@pytest.mark.parametrize("scale", [10, 13])
def test_triangle_counting_rmat(scale):
    L = mspgen.triangle_input(scale, 16, scale)
    dL = up(L)
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    for kind in ("auto", "hash", "maskidx", "inner"):
        for phase in (1, 2):
            C = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64", force_kind=kind, phase=phase)
            assert_same(C, R, "plus_pair_i64")
    C = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64", inner_ratio=4)
    assert_same(C, R, "plus_pair_i64")


@pytest.mark.parametrize("sr,vals", [("lor_land_bool", "u8"), ("plus_times_i32", "i32")])
def test_bfs_step(sr, vals):
    G = mspgen.rmat_graph(12, 8, 12)
    F, V, srcs, lv = mspgen.bfs_step_input(G, 512, seed=21, values=vals)
    for phase in (1, 2):
        run_and_check(G, F, V, True, sr, phase=phase)


def test_er_small_workload_full():
    """Erdos-Renyi n = 4096, 8 entries per row, U(0,1) FP64, normal mask."""
    A = mspgen.er(4096, 4096, 8.0, 101, "f64")
    B = mspgen.er(4096, 4096, 8.0, 102, "f64")
    M = mspgen.er(4096, 4096, 8.0, 103, None)
    for kind in ("auto", "hash", "maskidx", "dense", "inner"):
        run_and_check(A, B, M, False, "plus_times_f64", force_kind=kind)


def test_validation_rejects_bad_csr():
    m = msp()
    A = mspgen.er(50, 40, 5, 1, "f64")
    B = mspgen.er(40, 60, 5, 2, "f64")
    M = mspgen.er(50, 60, 5, 3, None)
    bad = mspgen.CSR(B.nrows, B.ncols, B.rowptr.copy(), B.colidx.copy(), B.values)
    r = int(np.argmax(np.diff(B.rowptr) >= 2))
    p = B.rowptr[r]
    bad.colidx[p], bad.colidx[p + 1] = bad.colidx[p + 1], bad.colidx[p]  # unsorted row
    with pytest.raises(m.MspError) as e:
        m.masked_spgemm(up(A, "plus_times_f64"), up(bad, "plus_times_f64"), up(M), validate=True)
    assert e.value.status == 3
    C = m.masked_spgemm(up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M), validate=True)
    assert_same(C, oracle.masked_spgemm(A, B, M, False, "plus_times_f64"), "plus_times_f64")


def test_plan_reuse_and_value_update():
    torch = torch_or_skip()
    m = msp()
    A = mspgen.er(500, 400, 6, 51, "f64")
    B = mspgen.er(400, 700, 6, 52, "f64")
    M = mspgen.er(500, 700, 30, 53, None)
    dA, dB, dM = up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M)
    with m.Plan(dA, dB, dM, semiring="plus_times_f64") as p:
        C1 = p.execute()
        C2 = p.execute()
        assert torch.equal(C1.colidx, C2.colidx)
        dA.values.mul_(2.0)  # same pattern, new values: the plan stays valid
        C3 = p.execute()
    A2 = A.with_values(A.values * 2.0)
    assert_same(C3, oracle.masked_spgemm(A2, B, M, False, "plus_times_f64"), "plus_times_f64")


def test_integer_results_repeat_bit_exact():
    torch = torch_or_skip()
    L = mspgen.triangle_input(12, 16, 3)
    dL = up(L)
    a = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64")
    b = msp().masked_spgemm(dL, dL, dL, semiring="plus_pair_i64", phase=2)
    assert torch.equal(a.rowptr, b.rowptr) and torch.equal(a.colidx, b.colidx) and torch.equal(a.values, b.values)


def test_reduce_semirings():
    torch = torch_or_skip()
    m = msp()
    dev = torch.device("cuda:0")
    x = torch.arange(1, 100001, dtype=torch.int64, device=dev)
    assert int(m.reduce(x, "plus_pair_i64").item()) == 100000 * 100001 // 2
    y = torch.rand(12345, dtype=torch.float64, device=dev)
    assert abs(float(m.reduce(y, "plus_times_f64").item()) - float(y.sum().item())) <= 1e-10
    z = torch.zeros(1000, dtype=torch.uint8, device=dev)
    assert int(m.reduce(z, "lor_land_bool").item()) == 0
    z[777] = 1
    assert int(m.reduce(z, "lor_land_bool").item()) == 1
    w = torch.full((1000,), 2**30, dtype=torch.int32, device=dev)
    assert int(m.reduce(w, "plus_times_i32").item()) == 0  # 1000 * 2^30 mod 2^32
    e = torch.zeros(0, dtype=torch.int64, device=dev)
    assert int(m.reduce(e, "plus_pair_i64").item()) == 0


@pytest.mark.parametrize("sr", SEMIRINGS)
@pytest.mark.parametrize("complement", [False, True])
@pytest.mark.parametrize("phase", [1, 2])
@pytest.mark.parametrize("ncols", [300, 3000])
def test_split_rows(sr, complement, phase, ncols):
    """Rows split over several workgroups by chunks of A's row (forced with a
    tiny threshold), merged through the global per-row accumulator."""
    A = mspgen.er(120, 400, 60.0, 61, {"plus_times_f64": "f64", "plus_pair_i64": "f64", "lor_land_bool": "u8",
                                      "plus_times_i32": "i32", "plus_times_i64": "i64"}[sr])
    B = mspgen.er(400, ncols, 25.0, 62, A.values is not None and {"plus_times_f64": "f64", "plus_pair_i64": "f64",
                  "lor_land_bool": "u8", "plus_times_i32": "i32", "plus_times_i64": "i64"}[sr] or None)
    M = mspgen.er(120, ncols, ncols / 6.0, 63, None)
    C, R = run_and_check(A, B, M, complement, sr, phase=phase, force_kind="dense", split_flops=300)


def long_a_rows(seed, m, k, sr):
    """Rows of A with 3 to 2500 entries: some below and some above the length
    at which a workgroup's waves take whole batches of 64 A entries (8
    batches), most with a ragged last batch."""
    rng = np.random.default_rng(seed)
    degs = rng.choice([3, 300, 511, 513, 700, 1500, 2500], size=m)
    rows = np.repeat(np.arange(m), degs)
    cols = np.concatenate([rng.choice(k, size=d, replace=False) for d in degs])
    A = mspgen.from_coo(m, k, rows, cols)
    return A.with_values(mspgen.random_values(A.nnz, VKIND[sr], rng))


@pytest.mark.parametrize("ncols", [400, 9000])
@pytest.mark.parametrize("kind", ["auto", "dense", "hash", "maskidx", "split"])
@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_pair_i64", "lor_land_bool", "plus_times_i32"])
@pytest.mark.parametrize("complement", [False, True])
def test_long_a_rows_claim_whole_batches(ncols, kind, sr, complement):
    """Long rows of A: the waves of a workgroup claim whole batches from a
    shared counter instead of sharing the windows of every batch. Forced
    kinds, both mask modes, and (n <= 512) rows split over workgroups whose
    chunks are long enough to claim batches too."""
    if kind == "split" and ncols > 512:
        pytest.skip("split rows are dense rows of at most 512 columns")
    if complement and kind in ("hash", "maskidx"):
        pytest.skip("a complemented mask takes only the dense and heap kinds")
    A = long_a_rows(31, 40, 6000, sr)
    B = mspgen.er(6000, ncols, 3.0, 32, VKIND[sr])
    M = mspgen.er(40, ncols, ncols / 8.0, 33, None)
    kw = dict(force_kind="dense", split_flops=2000) if kind == "split" else dict(force_kind=kind)
    for phase in (1, 2):
        run_and_check(A, B, M, complement, sr, phase=phase, **kw)


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_pair_i64"])
def test_long_a_rows_claim_whole_batches_in_batch(sr):
    """The same long rows of A in a batch of products (the batched kernels
    read each unit's operands from the descriptor table), replayed from a
    graph twice."""
    torch = torch_or_skip()
    m = msp()
    probs = []
    for t, (n, comp) in enumerate([(400, False), (9000, False), (400, True), (9000, True)]):
        A = long_a_rows(40 + t, 30, 5000, sr)
        B = mspgen.er(5000, n, 3.0, 50 + t, VKIND[sr])
        M = mspgen.er(30, n, n / 8.0, 60 + t, None)
        probs.append((A, B, M, comp))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
                for (A, B, M, c), C in zip(probs, b.results()):
                    assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)


def colliding_columns(count, bits, n):
    """The first `count` columns below n whose multiplicative hash (the odd
    constant 0x9E3779B1, top `bits` bits) is 0: keys that all share one home
    bucket, so the table's probe chains are as long as they can be."""
    j = np.arange(n, dtype=np.uint64)
    h = ((j * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - bits)
    cols = np.nonzero(h == 0)[0][:count]
    assert len(cols) == count
    return cols.astype(np.int64)


@pytest.mark.parametrize("keys", [200, 300, 512])
@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_pair_i64"])
def test_hash_keys_sharing_one_bucket(keys, sr):
    """Mask rows whose keys all hash to the same bucket (worst-case linear
    probing, both for inserting the keys and for looking up columns that are
    not keys), under the forced hash kind (one wave for at most 256 keys,
    a block above) and the automatic choice."""
    rng = np.random.default_rng(keys)
    n, k, m = 1 << 18, 400, 12
    hot = colliding_columns(keys, 8, n)
    M = mspgen.from_coo(m, n, np.repeat(np.arange(m), keys), np.tile(hot, m))
    # rows of B mix key columns (hits) with other columns that often share their home bucket
    near = colliding_columns(keys + 400, 8, n)[keys:]
    rows, cols = [], []
    for r in range(k):
        c = np.unique(np.concatenate([rng.choice(hot, 6, replace=False), rng.choice(near, 6, replace=False),
                                      rng.integers(0, n, 4)]))
        rows.append(np.full(len(c), r))
        cols.append(c)
    B = mspgen.from_coo(k, n, np.concatenate(rows), np.concatenate(cols))
    B = B.with_values(mspgen.random_values(B.nnz, VKIND[sr], rng))
    A = mspgen.er(m, k, 60.0, keys + 1, VKIND[sr])
    for kind in ("hash", "auto"):
        for phase in (1, 2):
            run_and_check(A, B, M, False, sr, phase=phase, force_kind=kind)


def test_split_rows_in_batch():
    torch = torch_or_skip()
    m = msp()
    sr = "plus_times_i32"
    probs = []
    for t in range(3):
        A = mspgen.er(90, 300, 50.0, 70 + t, "i32")
        B = mspgen.er(300, 500, 30.0, 80 + t, "i32")
        M = mspgen.er(90, 500, 60.0, 90 + t, None)
        probs.append((A, B, M, t % 2 == 1))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr, split_flops=200) as b:
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
            for (A, B, M, c), C in zip(probs, b.results()):
                assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)


def test_reduce_csr_reads_the_count_on_the_device():
    torch = torch_or_skip()
    m = msp()
    L = mspgen.triangle_input(12, 16, 7)
    dL = up(L)
    with m.Plan(dL, dL, dL, semiring="plus_pair_i64") as p:
        cap = max(p.upper_bound, 1)
        dev = dL.rowptr.device
        rp = torch.empty(L.nrows + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(cap, dtype=torch.int32, device=dev)
        v = torch.full((cap,), 7, dtype=torch.int64, device=dev)  # entries past nnz(C) must not count
        assert p.execute_into(rp, ci, v, cap) == -1
        got = m.reduce_csr(rp, L.nrows, v, "plus_pair_i64")
        n = int(rp[-1].item())
        assert n < cap
        assert int(got.item()) == int(m.reduce(v[:n], "plus_pair_i64").item())
        R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
        assert int(got.item()) == int(R.values.sum())
        # the count is clamped to the length of `values`
        assert int(m.reduce_csr(rp, L.nrows, v[:5], "plus_pair_i64").item()) == int(v[:5].sum().item())


def test_timing_session_without_per_execution_sync():
    torch = torch_or_skip()
    m = msp()
    A, B, M = rand_problem(31, 3000, 2000, 4000, 6.0, 9.0, 40.0, "plus_times_f64")
    R = oracle.masked_spgemm(A, B, M, False, "plus_times_f64")
    dA, dB, dM = up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M)
    T = m.Timing()
    stage = np.zeros(len(m.STAGE_NAMES))
    with m.Plan(dA, dB, dM, semiring="plus_times_f64") as p:
        cap = max(p.upper_bound, 1)
        outs = []
        for _ in range(3):
            rp = torch.empty(A.nrows + 1, dtype=torch.int64, device="cuda")
            ci = torch.empty(cap, dtype=torch.int32, device="cuda")
            v = torch.empty(cap, dtype=torch.float64, device="cuda")
            p.execute_timed(rp, ci, v, cap, T)
            outs.append((rp, ci, v))
        T.collect(stage)
        used = [b for b, k in enumerate(m.BIN_NAMES) if p.bin_units[k] > 0]
    # (a small heap bin runs inside the mask-indexed launch and has no time of its own)
    assert used and all(stage[b] > 0 for b in used if not m.BIN_NAMES[b].startswith("heap"))
    assert stage[m.STAGE_NAMES.index("compact")] > 0 and stage[m.STAGE_NAMES.index("scan")] > 0
    again = T.collect(np.zeros(len(m.STAGE_NAMES)))  # the session was emptied by the first collect
    assert not again.any()
    for rp, ci, v in outs:
        n = int(rp[-1].item())
        assert_same(msp().DeviceCSR(A.nrows, B.ncols, rp, ci[:n], v[:n]), R, "plus_times_f64")
    T.close()


@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("rot", [0, 1, 2, 3, 4])
def test_kind_table_per_row_class(comp, rot):
    """Every row class forced to a kind by the table (kinds rotating over
    the classes); entries that do not fit a row (complemented masks,
    oversized heap rows) fall back to the rules. Same result as the oracle."""
    m = msp()
    sr = "plus_times_f64"
    A, B, M = rand_problem(90 + rot, 700, 500, 6000, 6.0, 7.0, 60.0, sr)
    kinds = ["dense", "hash", "maskidx", "inner", "heap"]
    table = {c: kinds[(c + rot) % 5] for c in range(144)}
    C = m.masked_spgemm(up(A, sr), up(B, sr), up(M), complement=comp, semiring=sr, kind_table=table)
    assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)


@pytest.mark.parametrize("sr", ["plus_times_i32", "lor_land_bool", "plus_times_f64"])
def test_narrow_dense_rows_on_a_block(sr):
    """Dense rows of a matrix of at most 512 columns run on a block only
    above 32 x block_flops products: a small block_flops (and no split)
    sends the heavy rows there, under both mask modes."""
    m = msp()
    A, B, M = rand_problem(97, 900, 700, 480, 30.0, 40.0, 120.0, sr)
    for comp in (False, True):
        with m.Plan(up(A, sr), up(B, sr), up(M), complement=comp, semiring=sr, force_kind="dense",
                    block_flops=36, split_flops=0) as p:
            assert p.bin_units["dense_block_narrow"] > 0 and p.bin_units["dense_wave"] > 0
            C = p.execute()
        assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)
