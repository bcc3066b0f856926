"""Caller-owned workspaces through the C-ABI: size checks that refuse short
buffers before any kernel runs, the capacity check of the two-phase numeric
step, the one-shot call in one workspace, and one plan executed with two
workspaces on two streams."""
import ctypes

import numpy as np
import pytest

import mspgen
import oracle
from tests.gpu_util import assert_same, msp, rand_problem, torch_or_skip, up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_or_skip()


def _lib():
    from paper_2111_09947_amd import _lib as L
    return L.load(), L


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_short_execution_workspace_is_refused_before_any_kernel():
    import torch
    m = msp()
    lib, L = _lib()
    A, B, M = rand_problem(41, 300, 200, 400, 5.0, 6.0, 30.0, "plus_times_f64")
    with m.Plan(up(A, "plus_times_f64"), up(B, "plus_times_f64"), up(M), semiring="plus_times_f64") as p:
        cap = p.upper_bound
        rp = torch.full((p.nrows + 1,), -7, dtype=torch.int64, device="cuda:0")
        ci = torch.empty(cap, dtype=torch.int32, device="cuda:0")
        v = torch.empty(cap, dtype=torch.float64, device="cuda:0")
        out = L.MspCsrOut(p.nrows, p.ncols, cap, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
        ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device="cuda:0")
        st = lib.msp_execute(p._h, ctypes.byref(out), None, ctypes.c_void_p(ws.data_ptr()), p.workspace_bytes - 1,
                             _stream())
        assert st == 5 and b"execution workspace" in lib.msp_last_error()
        torch.cuda.synchronize()
        assert bool((rp == -7).all()), "a kernel wrote the output before the size check"
        # the full size runs
        n = ctypes.c_int64(0)
        st = lib.msp_execute(p._h, ctypes.byref(out), ctypes.byref(n), ctypes.c_void_p(ws.data_ptr()),
                             p.workspace_bytes, _stream())
        assert st == 0
        R = oracle.masked_spgemm(A, B, M, False, "plus_times_f64")
        assert n.value == R.nnz
        assert_same(m.DeviceCSR(p.nrows, p.ncols, rp, ci[:n.value], v[:n.value]), R, "plus_times_f64")


def test_numeric_refuses_a_capacity_below_nnz():
    """msp_numeric checks C's capacity against nnz(C) even when msp_symbolic
    did not return it (it reads the count itself), before any kernel runs."""
    import torch
    m = msp()
    lib, L = _lib()
    A, B, M = rand_problem(43, 300, 200, 400, 5.0, 6.0, 30.0, "plus_pair_i64")
    R = oracle.masked_spgemm(A, B, M, False, "plus_pair_i64")
    assert R.nnz > 2
    with m.Plan(up(A), up(B), up(M), semiring="plus_pair_i64", phase=2) as p:
        ws = p.workspace()
        rp = torch.empty(p.nrows + 1, dtype=torch.int64, device="cuda:0")
        st = lib.msp_symbolic(p._h, ctypes.c_void_p(rp.data_ptr()), None, ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream())
        assert st == 0
        short = R.nnz - 1
        ci = torch.full((short,), -3, dtype=torch.int32, device="cuda:0")
        v = torch.full((short,), -3, dtype=torch.int64, device="cuda:0")
        out = L.MspCsrOut(p.nrows, p.ncols, short, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
        st = lib.msp_numeric(p._h, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream())
        assert st == 5 and b"nnz" in lib.msp_last_error()
        torch.cuda.synchronize()
        assert bool((ci == -3).all()) and bool((v == -3).all())
        # another workspace than symbolic's is refused
        ws2 = torch.empty_like(ws)
        ci = torch.empty(R.nnz, dtype=torch.int32, device="cuda:0")
        v = torch.empty(R.nnz, dtype=torch.int64, device="cuda:0")
        out = L.MspCsrOut(p.nrows, p.ncols, R.nnz, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
        st = lib.msp_numeric(p._h, ctypes.byref(out), ctypes.c_void_p(ws2.data_ptr()), ws2.numel(), _stream())
        assert st == 1
        # the exact capacity runs
        st = lib.msp_numeric(p._h, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream())
        assert st == 0
        assert_same(m.DeviceCSR(p.nrows, p.ncols, rp, ci, v), R, "plus_pair_i64")


@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("phase", [1, 2])
def test_one_shot_in_one_workspace(comp, phase):
    m = msp()
    sr = "plus_times_i32"
    A, B, M = rand_problem(45 + phase, 257, 300, 9000, 7.0, 9.0, 60.0, sr)
    C, need = m.one_shot(up(A, sr), up(B, sr), up(M), complement=comp, semiring=sr, phase=phase)
    R = oracle.masked_spgemm(A, B, M, comp, sr)
    assert_same(C, R, sr)
    with m.Plan(up(A, sr), up(B, sr), up(M), complement=comp, semiring=sr, phase=phase) as p:
        assert need == p.plan_workspace_bytes + p.workspace_bytes


def test_one_plan_two_workspaces_two_streams():
    """Executions of one plan with different execution workspaces are
    independent: two streams run the same plan at once into two outputs."""
    import torch
    m = msp()
    sr = "plus_times_f64"
    A, B, M = rand_problem(47, 2000, 1500, 3000, 12.0, 10.0, 80.0, sr)
    R = oracle.masked_spgemm(A, B, M, False, sr)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with m.Plan(up(A, sr), up(B, sr), up(M), semiring=sr) as p:
        torch.cuda.synchronize()
        outs = []
        for s in (s1, s2):
            with torch.cuda.stream(s):
                ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device="cuda:0")
                rp = torch.empty(p.nrows + 1, dtype=torch.int64, device="cuda:0")
                ci = torch.empty(max(p.upper_bound, 1), dtype=torch.int32, device="cuda:0")
                v = torch.empty(max(p.upper_bound, 1), dtype=torch.float64, device="cuda:0")
                lib, L = _lib()
                out = L.MspCsrOut(p.nrows, p.ncols, p.upper_bound, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
                st = lib.msp_execute(p._h, ctypes.byref(out), None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     ctypes.c_void_p(s.cuda_stream))
                assert st == 0
                outs.append((rp, ci, v, ws))
        torch.cuda.synchronize()
        for rp, ci, v, _ in outs:
            n = int(rp[-1].item())
            assert_same(m.DeviceCSR(p.nrows, p.ncols, rp, ci[:n], v[:n]), R, sr)


def test_iterated_products_take_memory_from_the_caller():
    """k-truss and BC take every buffer from the binding's allocator and give
    all of it back."""
    m = msp()
    G = mspgen.rmat_graph(10, 8, 3)
    T, info = m.ktruss(up(G), 4)
    assert info["peak_device_bytes"] > 0
    bc, binfo = m.bc_batch(up(G), np.arange(16))
    assert binfo["peak_device_bytes"] > 0


def test_plans_and_batches_free_their_memory_without_the_cycle_collector():
    """A Plan or Batch dropped by the caller releases its workspaces (and a
    batch its outputs) at once: no reference cycle keeps them until the
    cyclic garbage collector runs."""
    import gc
    import weakref
    m = msp()
    sr = "plus_times_f64"
    A, B, M = rand_problem(44, 300, 200, 400, 5.0, 6.0, 30.0, sr)
    d = (up(A, sr), up(B, sr), up(M))
    gc.disable()
    try:
        p = m.Plan(*d, semiring=sr)
        p.execute()
        ref = weakref.ref(p)
        del p
        assert ref() is None
        b = m.Batch([d + (False,), d + (False,)], semiring=sr)
        b.bind_new_outputs()
        b.execute()
        ref = weakref.ref(b)
        del b
        assert ref() is None
    finally:
        gc.enable()
