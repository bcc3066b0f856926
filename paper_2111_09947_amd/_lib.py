"""ctypes declarations for libmsp.so (include/msp.h)."""
from __future__ import annotations

import ctypes
import os

# MSP_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MSP_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmsp.so")

c_i32, c_i64, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class MspCsr(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("nnz", c_i64),
                ("rowptr", c_vp), ("colidx", c_vp), ("values", c_vp)]


class MspCsrOut(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("capacity", c_i64),
                ("rowptr", c_vp), ("colidx", c_vp), ("values", c_vp)]


class MspOptions(ctypes.Structure):
    _fields_ = [("phase", c_i32), ("force_kind", c_i32), ("validate", c_i32),
                ("inner_ratio", c_i32), ("b_transpose", ctypes.POINTER(MspCsr)),
                ("maskidx_max", c_i32), ("heap_flops", c_i32), ("block_flops", c_i64), ("split_flops", c_i64),
                ("kind_table", ctypes.POINTER(ctypes.c_int8))]


ROW_BUCKETS = 12
KIND_CLASSES = ROW_BUCKETS * ROW_BUCKETS


class MspPlanInfo(ctypes.Structure):
    _fields_ = [("upper_bound", c_i64), ("products", c_i64), ("units", c_i64),
                ("staging", c_i64), ("mask_nnz", c_i64), ("kind_units", c_i64 * 8),
                ("bin_units", c_i64 * 16)]


class MspBcInfo(ctypes.Structure):
    _fields_ = [("levels", c_i64), ("frontier_nnz", c_i64), ("forward_products", c_i64),
                ("backward_products", c_i64), ("forward_ms", ctypes.c_double), ("backward_ms", ctypes.c_double)]


class MspKtrussInfo(ctypes.Structure):
    _fields_ = [("iterations", c_i64), ("products", c_i64), ("ms", ctypes.c_double)]


BIN_NAMES = ["dense_wave", "dense_block", "hash_wave", "hash_block", "maskidx_wave", "maskidx_block",
             "inner_wave", "dense_block_narrow", "dense_split", "heap_lane", "heap_lane_long_mask",
             "maskidx_packed", "sort_block"]
STAGE_NAMES = BIN_NAMES + [f"bin{b}" for b in range(len(BIN_NAMES), 16)] + [
    "symbolic", "scan", "rowptr", "compact", "split_emit", "place"]
NSTAGES = len(STAGE_NAMES)


class MspProblem(ctypes.Structure):
    _fields_ = [("A", MspCsr), ("B", MspCsr), ("M", MspCsr), ("complement", c_i32), ("reserved", c_i32)]


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, c_vp, ctypes.c_size_t, c_vp)
RELEASE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp, c_vp)


class MspAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", c_vp)]


c_sz = ctypes.c_size_t
P_sz = ctypes.POINTER(ctypes.c_size_t)
P_csr = ctypes.POINTER(MspCsr)
P_out = ctypes.POINTER(MspCsrOut)
P_opt = ctypes.POINTER(MspOptions)

# every symbol include/msp.h declares, with its ctypes signature
SIGNATURES = {
    "msp_options_default": (None, [P_opt]),
    "msp_plan_workspace_size": (ctypes.c_int, [P_csr, P_csr, P_csr, ctypes.c_int, ctypes.c_int, P_opt, P_sz]),
    "msp_plan_create": (ctypes.c_int, [ctypes.POINTER(c_vp), P_csr, P_csr, P_csr, ctypes.c_int, ctypes.c_int,
                                       P_opt, c_vp, c_sz, c_vp]),
    "msp_workspace_size": (ctypes.c_int, [c_vp, P_sz]),
    "msp_plan_info": (ctypes.c_int, [c_vp, ctypes.POINTER(MspPlanInfo)]),
    "msp_symbolic": (ctypes.c_int, [c_vp, c_vp, ctypes.POINTER(c_i64), c_vp, c_sz, c_vp]),
    "msp_numeric": (ctypes.c_int, [c_vp, P_out, c_vp, c_sz, c_vp]),
    "msp_execute": (ctypes.c_int, [c_vp, P_out, ctypes.POINTER(c_i64), c_vp, c_sz, c_vp]),
    "msp_execute_profiled": (ctypes.c_int, [c_vp, P_out, ctypes.POINTER(c_i64), c_vp, c_sz,
                                            ctypes.POINTER(ctypes.c_double), c_vp]),
    "msp_timing_create": (ctypes.c_int, [ctypes.POINTER(c_vp), ctypes.c_int32, ctypes.c_uint32]),
    "msp_execute_timed": (ctypes.c_int, [c_vp, P_out, ctypes.POINTER(c_i64), c_vp, c_sz, c_vp, c_vp]),
    "msp_timing_collect": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_double)]),
    "msp_timing_destroy": (None, [c_vp]),
    "msp_plan_row_bins": (ctypes.c_int, [c_vp, c_vp, c_vp]),
    "msp_plan_destroy": (None, [c_vp]),
    "msp_masked_spgemm": (ctypes.c_int, [P_csr, P_csr, P_csr, ctypes.c_int, ctypes.c_int, P_opt, P_out,
                                         ctypes.POINTER(c_i64), c_vp, c_sz, P_sz, c_vp]),
    "msp_masked_spgemm_noalloc": (ctypes.c_int, [P_csr, P_csr, P_csr, ctypes.c_int, ctypes.c_int, P_opt, P_out,
                                                 ctypes.POINTER(c_i64), P_sz, c_vp]),
    "msp_upper_bound": (ctypes.c_int, [P_csr, P_csr, P_csr, ctypes.c_int, ctypes.POINTER(c_i64), c_vp, c_sz, c_vp]),
    "msp_reduce": (ctypes.c_int, [c_vp, c_i64, ctypes.c_int, c_vp, c_vp, c_sz, c_vp]),
    "msp_reduce_workspace_size": (ctypes.c_int, [P_sz]),
    "msp_reduce_csr": (ctypes.c_int, [c_vp, c_i64, c_vp, c_i64, ctypes.c_int, c_vp, c_vp, c_sz, c_vp]),
    "msp_batch_workspace_size": (ctypes.c_int, [ctypes.POINTER(MspProblem), c_i64, ctypes.c_int, P_opt, P_sz]),
    "msp_batch_create": (ctypes.c_int, [ctypes.POINTER(c_vp), ctypes.POINTER(MspProblem), c_i64, ctypes.c_int,
                                        P_opt, c_vp, c_sz, c_vp]),
    "msp_batch_count": (c_i64, [c_vp]),
    "msp_batch_info": (ctypes.c_int, [c_vp, c_i64, ctypes.POINTER(MspPlanInfo)]),
    "msp_batch_bind": (ctypes.c_int, [c_vp, P_out, c_vp, c_sz, c_vp]),
    "msp_batch_execute": (ctypes.c_int, [c_vp, c_vp]),
    "msp_batch_execute_timed": (ctypes.c_int, [c_vp, c_vp, c_vp]),
    "msp_batch_graph_launch": (ctypes.c_int, [c_vp, c_vp]),
    "msp_batch_nnz": (ctypes.c_int, [c_vp, ctypes.POINTER(c_i64), c_vp]),
    "msp_ktruss": (ctypes.c_int, [P_csr, ctypes.c_int32, c_vp, c_vp, c_vp, ctypes.POINTER(c_i64),
                                  ctypes.POINTER(MspKtrussInfo), ctypes.POINTER(MspAllocator), c_vp]),
    "msp_bc_batch": (ctypes.c_int, [P_csr, c_vp, c_i64, c_vp, ctypes.POINTER(MspBcInfo),
                                    ctypes.POINTER(MspAllocator), c_vp]),
    "msp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "msp_last_error": (ctypes.c_char_p, []),
    "msp_version": (ctypes.c_int, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Loads the in-tree libmsp.so; raises if it has not been built. There is
    no fallback: the masked product runs only in the HIP library."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2111_09947_amd.build or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
