"""GPU parity of the packed mask-indexed bin (eight lanes per row, eight rows
per wave), which takes rows with a normal mask row of at most 16 entries, at
most 256 products and at most 32 entries in the row of A when the binner
chooses automatically. Each case checks that the bin ran and compares the
result with the oracle: patterns and integer values bit-exact, FP64 within
1e-12 relative."""
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


def _plan_check(A, B, M, sr, complement=False, phase=1):
    m = msp()
    with m.Plan(up(A, sr), up(B, sr), up(M), complement, sr, phase=phase) as p:
        C = p.execute()
        bins = dict(p.bin_units)
    assert_same(C, oracle.masked_spgemm(A, B, M, complement, sr), sr)
    return bins


@pytest.mark.parametrize("phase", [1, 2])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_er_rows_run_packed(sr, phase):
    """Erdos-Renyi n = 4096 with 8 entries per row (A, B and the mask): nearly
    every row is packed."""
    A = mspgen.er(4096, 4096, 8.0, 101, VKIND[sr])
    B = mspgen.er(4096, 4096, 8.0, 102, VKIND[sr])
    M = mspgen.er(4096, 4096, 8.0, 103, None)
    bins = _plan_check(A, B, M, sr, phase=phase)
    assert bins["maskidx_packed"] > 0.9 * sum(bins.values())


def _boundary_problem(sr, seed=3):
    """Rows built to sit on both sides of each packing limit. B row b has b % 10
    entries (so some are empty). Row types (cycled): 32 entries of A with 256
    products and 16 mask entries (packed); 33 entries of A (not packed); 32
    entries with 257 products (not packed); 17 mask entries (not packed); a few
    entries of A of which most have empty B rows, one mask entry (packed); mask
    columns 0 and n - 1 among the keys (packed). About half of every mask row
    is drawn from the row's own product columns, so that rows have hits, and
    several A entries reach the same key, so that hits are summed."""
    rng = np.random.default_rng(seed)
    n, k = 3000, 2000
    blen = np.arange(k) % 10
    brows, bcols = [], []
    for b in range(k):
        c = np.sort(rng.choice(n, size=blen[b], replace=False))
        brows.append(np.full(blen[b], b))
        bcols.append(c)
    B = mspgen.from_coo(k, n, np.concatenate(brows), np.concatenate(bcols))
    by_len = {L: np.nonzero(blen == L)[0] for L in range(10)}
    arows, acols, mrows, mcols = [], [], [], []
    m = 180
    for i in range(m):
        t = i % 6
        if t == 0:
            ent = rng.choice(by_len[8], size=32, replace=False)                       # 256 products
            mlen = 16
        elif t == 1:
            ent = rng.choice(by_len[3], size=33, replace=False)                       # 33 entries of A
            mlen = 8
        elif t == 2:
            ent = np.concatenate([rng.choice(by_len[8], size=31, replace=False), rng.choice(by_len[9], size=1)])
            mlen = 12                                                                # 257 products
        elif t == 3:
            ent = rng.choice(by_len[5], size=6, replace=False)
            mlen = 17                                                                # 17 mask entries
        elif t == 4:
            ent = np.concatenate([rng.choice(by_len[0], size=4, replace=False), rng.choice(by_len[2], size=1)])
            mlen = 1                                                                 # mostly empty B rows
        else:
            ent = rng.choice(by_len[7], size=5, replace=False)
            mlen = 14
        ent = np.sort(ent)
        arows.append(np.full(len(ent), i))
        acols.append(ent)
        prod = np.unique(np.concatenate([bcols[b] for b in ent]) if len(ent) else np.zeros(0, np.int64))
        hit = rng.choice(prod, size=min(len(prod), mlen // 2), replace=False) if len(prod) else np.zeros(0, np.int64)
        extra = [0, n - 1] if t == 5 else []
        rest = np.setdiff1d(np.arange(n), np.concatenate([hit, extra]).astype(np.int64))
        fill = rng.choice(rest, size=mlen - len(hit) - len(extra), replace=False)
        mc = np.unique(np.concatenate([hit, extra, fill]).astype(np.int64))
        assert len(mc) == mlen
        mrows.append(np.full(mlen, i))
        mcols.append(mc)
    A = mspgen.from_coo(m, k, np.concatenate(arows), np.concatenate(acols))
    M = mspgen.from_coo(m, n, np.concatenate(mrows), np.concatenate(mcols))
    vk = VKIND[sr]
    A = A.with_values(mspgen.random_values(A.nnz, vk, np.random.default_rng(seed + 10)))
    B = B.with_values(mspgen.random_values(B.nnz, vk, np.random.default_rng(seed + 20)))
    return A, B, M


@pytest.mark.parametrize("phase", [1, 2])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_packing_limits(sr, phase):
    A, B, M = _boundary_problem(sr)
    bins = _plan_check(A, B, M, sr, phase=phase)
    packed = bins["maskidx_packed"]
    assert packed == 90, bins  # the three packed row types, 30 rows each
    assert sum(bins.values()) - packed > 0


def test_complemented_mask_is_never_packed():
    A = mspgen.er(4096, 4096, 8.0, 101, "f64")
    B = mspgen.er(4096, 4096, 8.0, 102, "f64")
    M = mspgen.er(4096, 4096, 8.0, 103, None)
    bins = _plan_check(A, B, M, "plus_times_f64", complement=True)
    assert bins["maskidx_packed"] == 0


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_i32"])
def test_packed_rows_in_a_batch(sr):
    """Products of different sizes in one batch (the groups of one wave can
    belong to different products), replayed from a captured graph twice."""
    torch = torch_or_skip()
    m = msp()
    probs = []
    for t, (n, d) in enumerate([(4096, 8.0), (1000, 4.0), (20000, 6.0), (777, 10.0)]):
        A = mspgen.er(n, n, d, 300 + 3 * t, VKIND[sr])
        B = mspgen.er(n, n, d, 301 + 3 * t, VKIND[sr])
        M = mspgen.er(n, n, d, 302 + 3 * t, None)
        probs.append((A, B, M, False))
    A, B, M = _boundary_problem(sr, seed=9)
    probs.append((A, B, M, False))
    dev = [(up(A, sr), up(B, sr), up(M), c) for (A, B, M, c) in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with m.Batch(dev, semiring=sr) as b:
            assert b.bin_units["maskidx_packed"] > 0
            b.bind_new_outputs()
            for _ in range(2):
                b.graph_launch()
                for (A, B, M, c), C in zip(probs, b.results()):
                    assert_same(C, oracle.masked_spgemm(A, B, M, c, sr), sr)
