"""GPU parity of the dense kernels reading B's column indices from the 16-bit
copy that an execution makes when B has at most 512 columns and its rows are
re-read at least 4 times over: every semiring, both phases, both mask modes,
column 511 present, a B whose column indices start at an address that is not
16-byte aligned (the copy's element-wise path), split rows, and a plan run
twice with B's column indices changed in between (the copy is remade by each
execution). Patterns and integer values bit-exact, FP64 within 1e-12
relative."""
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


def _problem(sr, seed, m=2000, k=600, n=512, da=24.0, db=40.0, dm=60.0):
    A = mspgen.er(m, k, da, seed, VKIND[sr])
    B = mspgen.er(k, n, db, seed + 1, VKIND[sr])
    M = mspgen.er(m, n, dm, seed + 2, None)
    return A, B, M


@pytest.mark.parametrize("phase", [1, 2])
@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_dense_rows_with_16bit_columns(sr, comp, phase):
    A, B, M = _problem(sr, 400 + SEMIRINGS.index(sr))
    assert (B.colidx == 511).any()
    m = msp()
    with m.Plan(up(A, sr), up(B, sr), up(M), comp, sr, phase=phase, force_kind="dense") as p:
        assert p.bin_units["dense_wave"] > 0
        C = p.execute()
    assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)


def _misaligned(X, sr):
    """X on the GPU with its column indices one int32 past a 256-byte boundary."""
    torch = torch_or_skip()
    m = msp()
    d = up(X, sr)
    buf = torch.empty(X.nnz + 1, dtype=torch.int32, device=d.colidx.device)
    buf[1:].copy_(d.colidx)
    ci = buf[1:]
    assert ci.data_ptr() % 16 == 4
    return m.DeviceCSR(X.nrows, X.ncols, d.rowptr, ci, d.values)


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_i32", "lor_land_bool"])
def test_unaligned_b_columns(sr):
    A, B, M = _problem(sr, 420, da=30.0)
    m = msp()
    for comp in (False, True):
        C = m.masked_spgemm(up(A, sr), _misaligned(B, sr), up(M), complement=comp, semiring=sr)
        assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)


def test_split_rows_with_16bit_columns():
    """Rows past the split threshold run in chunks, each reading the copy."""
    sr = "plus_times_i64"
    A = mspgen.er(60, 3000, 900.0, 431, VKIND[sr])
    B = mspgen.er(3000, 300, 250.0, 432, VKIND[sr])
    M = mspgen.er(60, 300, 40.0, 433, None)
    m = msp()
    for comp in (False, True):
        with m.Plan(up(A, sr), up(B, sr), up(M), comp, sr, split_flops=65536) as p:
            assert p.bin_units["dense_split"] > 0
            C = p.execute()
        assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)


def test_plan_rerun_after_b_columns_change():
    """Same B row pointers, other column indices: the second execution of the
    plan reads the new columns."""
    torch = torch_or_skip()
    sr = "plus_times_f64"
    A, B, M = _problem(sr, 440)
    rng = np.random.default_rng(441)
    cols = np.concatenate([np.sort(rng.choice(B.ncols, size=int(B.rowptr[i + 1] - B.rowptr[i]), replace=False))
                           for i in range(B.nrows)]).astype(np.int32)
    B2 = mspgen.CSR(B.nrows, B.ncols, B.rowptr.copy(), cols, B.values.copy())
    m = msp()
    dB = up(B, sr)
    with m.Plan(up(A, sr), dB, up(M), False, sr) as p:
        assert p.bin_units["dense_wave"] > 0
        C1 = p.execute()
        assert_same(C1, oracle.masked_spgemm(A, B, M, False, sr), sr)
        dB.colidx.copy_(torch.from_numpy(cols).to(dB.colidx.device))
        C2 = p.execute()
        assert_same(C2, oracle.masked_spgemm(A, B2, M, False, sr), sr)
