"""msp_masked_spgemm_noalloc through the C-ABI: the one-shot product in the
library's fixed device scratch gives the same C as msp_masked_spgemm with a
caller workspace (and as the oracle), on consecutive calls that reuse the
scratch with a smaller second input; a product larger than the scratch is
refused with its size."""
import ctypes

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_same, msp, rand_problem, torch_or_skip, up

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_or_skip()


def _lib():
    from paper_2111_09947_amd import _lib as L
    return L.load(), L


def _noalloc(dA, dB, dM, comp, sr, cap, phase=1):
    """Calls msp_masked_spgemm_noalloc directly; returns (status, C, ws_needed)."""
    import torch
    m = msp()
    lib, L = _lib()
    dev = dA.rowptr.device
    rp = torch.full((dA.nrows + 1,), -7, dtype=torch.int64, device=dev)
    ci = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    v = torch.empty(max(cap, 1), dtype=m.out_dtype(sr), device=dev)
    vs = (m._view(dA, sr, "A"), m._view(dB, sr, "B"), m._view(dM, None, "M"))
    o = m.options(phase=phase)
    out = L.MspCsrOut(dA.nrows, dB.ncols, cap, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
    n = ctypes.c_int64(-1)
    need = ctypes.c_size_t(0)
    st = lib.msp_masked_spgemm_noalloc(*(ctypes.byref(x) for x in vs), int(comp), m.SEMIRINGS[sr], ctypes.byref(o),
                                       ctypes.byref(out), ctypes.byref(n), ctypes.byref(need),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    C = m.DeviceCSR(dA.nrows, dB.ncols, rp, ci[:max(n.value, 0)], v[:max(n.value, 0)])
    return st, C, need.value, n.value


def _compare(C, Cref, sr):
    """Same pattern, integer values identical, FP64 within 1e-12 relative."""
    rp, ci, v = C.to_host()
    rr, cr, vr = Cref.to_host()
    assert np.array_equal(rp, rr), "rowptr differs from msp_masked_spgemm"
    assert np.array_equal(ci, cr), "colidx differs from msp_masked_spgemm"
    if sr == "plus_times_f64":
        assert np.all(np.abs(v - vr) <= 1e-12 * np.abs(vr)), "fp64 values differ from msp_masked_spgemm"
    else:
        assert np.array_equal(v, vr), "values differ from msp_masked_spgemm"


@pytest.mark.parametrize("sr,comp,phase", [("plus_times_f64", False, 1), ("plus_pair_i64", True, 1),
                                           ("plus_times_i32", False, 2)])
def test_noalloc_matches_the_workspace_call_twice(sr, comp, phase):
    m = msp()
    # first a larger product, then a smaller one in the same scratch
    for seed, (rows, inner, cols, da, db, dm) in ((61, (3000, 2500, 2800, 8.0, 8.0, 40.0)),
                                                  (62, (400, 300, 350, 5.0, 6.0, 25.0))):
        A, B, M = rand_problem(seed, rows, inner, cols, da, db, dm, sr)
        dA, dB, dM = up(A, sr), up(B, sr), up(M)
        Cref, need_ws = m.one_shot(dA, dB, dM, complement=comp, semiring=sr, phase=phase)
        assert need_ws <= SCRATCH_BYTES
        # a capacity of 0 reports the bound (phase 1) or nnz(C) (phase 2), as msp_masked_spgemm does
        st, _, _, bound = _noalloc(dA, dB, dM, comp, sr, 0, phase)
        assert st == 5 and bound >= Cref.nnz
        st, C, need, nnz = _noalloc(dA, dB, dM, comp, sr, bound, phase)
        assert st == 0, _lib()[0].msp_last_error()
        assert need == need_ws
        assert nnz == Cref.nnz
        _compare(C, Cref, sr)
        assert_same(C, oracle.masked_spgemm(A, B, M, comp, sr), sr)


def test_noalloc_refuses_a_product_above_the_scratch():
    import torch
    sr = "plus_times_f64"
    A, B, M = rand_problem(63, 600_000, 600_000, 600_000, 4.0, 4.0, 16.0, sr)
    dA, dB, dM = up(A, sr), up(B, sr), up(M)
    st, C, need, _ = _noalloc(dA, dB, dM, False, sr, 1 << 20)
    assert st == 5
    assert need > SCRATCH_BYTES
    assert b"fixed scratch" in _lib()[0].msp_last_error()
    torch.cuda.synchronize()
    assert bool((C.rowptr == -7).all()), "the refused call wrote the output"
