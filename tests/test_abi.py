"""The C-ABI library: it loads, exports every symbol include/msp.h declares,
and its host-side argument checks return the documented status without
touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msp.h")


def _lib():
    from paper_2111_09947_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2111_09947_amd import build
        build.build()
    return L.load(), L


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib, L = _lib()
    names = _declared()
    assert "msp_masked_spgemm" in names and "msp_plan_create" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert set(L.SIGNATURES) == set(names)


def test_host_only_calls():
    lib, L = _lib()
    assert lib.msp_version() >= 100
    assert lib.msp_status_string(0) == b"ok"
    assert lib.msp_status_string(3) == b"invalid CSR"
    o = L.MspOptions()
    lib.msp_options_default(ctypes.byref(o))
    assert (o.phase, o.force_kind, o.validate, o.inner_ratio) == (1, -1, 0, 0)
    assert (o.maskidx_max, o.heap_flops, o.block_flops, o.split_flops) == (-1, -1, -1, -1)


def _csr(L, nrows, ncols, nnz=0, rowptr=1):
    return L.MspCsr(nrows, ncols, nnz, rowptr, 0 if nnz == 0 else 8, 0)


def test_argument_errors_need_no_gpu():
    lib, L = _lib()
    h = ctypes.c_void_p()
    A, B, M = _csr(L, 4, 5), _csr(L, 5, 6), _csr(L, 4, 6)
    # NULL operand
    st = lib.msp_plan_create(ctypes.byref(h), None, ctypes.byref(B), ctypes.byref(M), 0, 0, None, None)
    assert st == 1
    # dimension mismatch
    Bbad = _csr(L, 7, 6)
    st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(A), ctypes.byref(Bbad), ctypes.byref(M), 0, 0, None, None)
    assert st == 2 and b"A.ncols" in lib.msp_last_error()
    # unknown semiring
    st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(A), ctypes.byref(B), ctypes.byref(M), 0, 9, None, None)
    assert st == 1
    # complemented mask with a mask-keyed kind
    o = L.MspOptions()
    lib.msp_options_default(ctypes.byref(o))
    for kind in (1, 2, 3):
        o.force_kind = kind
        st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(A), ctypes.byref(B), ctypes.byref(M), 1, 0,
                                 ctypes.byref(o), None)
        assert st == 4
    # unknown kind
    o.force_kind = 5
    st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(A), ctypes.byref(B), ctypes.byref(M), 0, 0,
                             ctypes.byref(o), None)
    assert st == 1 and b"force_kind" in lib.msp_last_error()
    # bad phase
    o.force_kind = -1
    o.phase = 3
    st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(A), ctypes.byref(B), ctypes.byref(M), 0, 0,
                             ctypes.byref(o), None)
    assert st == 1
    # nnz > 0 with NULL colidx
    Anull = L.MspCsr(4, 5, 3, 1, 0, 0)
    st = lib.msp_plan_create(ctypes.byref(h), ctypes.byref(Anull), ctypes.byref(B), ctypes.byref(M), 0, 0, None, None)
    assert st == 1
    # reduce with negative length
    assert lib.msp_reduce(None, -1, 0, ctypes.c_void_p(8), None) == 1


def test_timing_and_csr_reduce_argument_errors():
    lib, L = _lib()
    assert lib.msp_timing_create(None, 0, 0) == 1
    h = ctypes.c_void_p()
    assert lib.msp_timing_create(ctypes.byref(h), -1, 0) == 1 and b"executions" in lib.msp_last_error()
    assert lib.msp_execute_timed(None, None, None, None, None) == 1
    assert lib.msp_timing_collect(None, None) == 1
    lib.msp_timing_destroy(None)  # accepted, does nothing
    assert lib.msp_reduce_csr(None, 5, None, 0, 1, None, None) == 1
    assert lib.msp_reduce_csr(ctypes.c_void_p(8), -1, None, 0, 1, None, None) == 1
    assert lib.msp_reduce_csr(ctypes.c_void_p(8), 5, None, 0, 9, ctypes.c_void_p(8), None) == 1  # semiring
    assert lib.msp_reduce_csr(ctypes.c_void_p(8), 5, None, 4, 1, ctypes.c_void_p(8), None) == 1  # values NULL
