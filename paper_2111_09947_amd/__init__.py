"""Masked sparse matrix-matrix products C = M .* (A B) on AMD MI355X.

Thin Python binding over the C-ABI library ``libmsp.so`` (include/msp.h):
it only marshals torch device tensors and the current HIP stream; every step
of the product runs in the library's HIP kernels. Importing works without a
GPU; calling needs the built library and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import functools
from typing import Optional

from . import _lib as L

SEMIRINGS = {
    "plus_times_f64": 0,
    "plus_pair_i64": 1,
    "lor_land_bool": 2,
    "plus_times_i32": 3,
    "plus_times_i64": 4,
}
BIN_NAMES = L.BIN_NAMES
STAGE_NAMES = L.STAGE_NAMES
KINDS = {None: -1, "auto": -1, "dense": 0, "hash": 1, "maskidx": 2, "inner": 3, "heap": 4}
STATUS = {0: "MSP_OK", 1: "MSP_ERR_INVALID_ARGUMENT", 2: "MSP_ERR_DIMENSION_MISMATCH",
          3: "MSP_ERR_INVALID_CSR", 4: "MSP_ERR_UNSUPPORTED", 5: "MSP_ERR_INSUFFICIENT_CAPACITY",
          6: "MSP_ERR_OUT_OF_MEMORY", 7: "MSP_ERR_DEVICE"}


class MspError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = L.load()
        detail = lib.msp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)} ({detail})")
        self.status = status


def _torch():
    import torch
    return torch


def in_dtype(semiring: str):
    t = _torch()
    return {"plus_times_f64": t.float64, "plus_pair_i64": None, "lor_land_bool": t.uint8,
            "plus_times_i32": t.int32, "plus_times_i64": t.int64}[semiring]


def out_dtype(semiring: str):
    t = _torch()
    return {"plus_times_f64": t.float64, "plus_pair_i64": t.int64, "lor_land_bool": t.uint8,
            "plus_times_i32": t.int32, "plus_times_i64": t.int64}[semiring]


@dataclasses.dataclass
class DeviceCSR:
    """CSR on the GPU: int64 rowptr, int32 colidx (sorted, unique per row),
    optional values."""

    nrows: int
    ncols: int
    rowptr: "object"
    colidx: "object"
    values: "Optional[object]" = None

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    @staticmethod
    def from_host(X, device="cuda", values_dtype=None) -> "DeviceCSR":
        """Upload a host CSR (numpy arrays: rowptr, colidx, values or None)."""
        t = _torch()
        rp = t.from_numpy(X.rowptr).to(device=device, dtype=t.int64)
        ci = t.from_numpy(X.colidx).to(device=device, dtype=t.int32)
        v = None
        if X.values is not None and values_dtype is not None:
            v = t.from_numpy(X.values).to(device=device, dtype=values_dtype)
        return DeviceCSR(X.nrows, X.ncols, rp.contiguous(), ci.contiguous(), v)

    def to_host(self):
        """(rowptr, colidx, values) as numpy arrays."""
        return (self.rowptr.cpu().numpy(), self.colidx.cpu().numpy(),
                None if self.values is None else self.values.cpu().numpy())


def _view(X: DeviceCSR, semiring: str, name: str) -> L.MspCsr:
    t = _torch()
    if X.rowptr.dtype != t.int64 or X.colidx.dtype != t.int32:
        raise TypeError(f"{name}: rowptr must be int64 and colidx int32")
    if not (X.rowptr.is_cuda and X.colidx.is_cuda):
        raise ValueError(f"{name}: tensors must be on the GPU")
    if not (X.rowptr.is_contiguous() and X.colidx.is_contiguous()):
        raise ValueError(f"{name}: tensors must be contiguous")
    vals = 0
    want = in_dtype(semiring) if semiring is not None else None
    if X.values is not None and want is not None:
        if X.values.dtype != want:
            raise TypeError(f"{name}: values must be {want} for {semiring}")
        if not X.values.is_contiguous():
            raise ValueError(f"{name}: values must be contiguous")
        vals = X.values.data_ptr()
    return L.MspCsr(X.nrows, X.ncols, X.colidx.numel(), X.rowptr.data_ptr(),
                    X.colidx.data_ptr() if X.colidx.numel() else 0, vals)


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _check(st: int, where: str):
    if st != 0:
        raise MspError(st, where)


def _workspace(nbytes: int, device):
    """A caller-owned device workspace of nbytes bytes (a torch tensor; the
    caching allocator's blocks are 512-byte aligned, the library needs 256)."""
    t = _torch()
    ws = t.empty(max(int(nbytes), 1), dtype=t.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


_WIDTH = {}


def _carve(alloc, n: int, dtype):
    """n elements of dtype from a byte allocator (alloc(nbytes) -> uint8
    device tensor starting on a 256-byte boundary)."""
    width = _WIDTH.get(dtype)
    if width is None:
        width = _WIDTH[dtype] = _torch().empty(0, dtype=dtype).element_size()
    nb = max(int(n), 1) * width
    return alloc(nb)[:nb].view(dtype)


class _Slab:
    """A byte allocator over one device tensor: consecutive slices, each on a
    256-byte boundary (the views keep the whole tensor alive)."""

    def __init__(self, nbytes: int, device):
        t = _torch()
        self.buf = t.empty(max(int(nbytes), 1), dtype=t.uint8, device=device)
        self.off = 0

    @staticmethod
    def size(n: int) -> int:
        return (max(int(n), 1) + 255) // 256 * 256

    def __call__(self, nbytes: int):
        n = self.size(nbytes)
        if self.off + n > self.buf.numel():
            raise RuntimeError("output slab exhausted")
        v = self.buf[self.off:self.off + n]
        self.off += n
        return v


class _TorchAllocator:
    """msp_allocator over torch device tensors: the library's iterated
    products (betweenness centrality, k-truss) take every working buffer from
    here, on the current stream, and release it in stream order."""

    def __init__(self, device):
        self.device = device
        self.held = {}
        self.peak = 0
        self.in_use = 0
        self._alloc = L.ALLOC_FN(self._on_alloc)
        self._release = L.RELEASE_FN(self._on_release)
        self.struct = L.MspAllocator(self._alloc, self._release, None)

    def _on_alloc(self, ctx, nbytes, stream):
        try:
            t = _workspace(nbytes, self.device)
        except Exception:  # out of memory: the library reports MSP_ERR_OUT_OF_MEMORY
            return None
        self.held[t.data_ptr()] = t
        self.in_use += t.numel()
        self.peak = max(self.peak, self.in_use)
        return t.data_ptr()

    def _on_release(self, ctx, ptr, stream):
        t = self.held.pop(ptr, None)
        if t is not None:
            self.in_use -= t.numel()


def kind_table_array(table):
    """A kind table (a sequence of KIND_CLASSES kind names or ids, or a
    {(flops_bucket, mask_bucket): kind} dict; None entries and missing classes
    keep the automatic rules) as the C array msp_options.kind_table reads."""
    arr = (ctypes.c_int8 * L.KIND_CLASSES)(*([-1] * L.KIND_CLASSES))
    items = table.items() if isinstance(table, dict) else enumerate(table)
    for key, kind in items:
        c = key[0] * L.ROW_BUCKETS + key[1] if isinstance(key, tuple) else int(key)
        arr[c] = KINDS[kind] if (kind is None or isinstance(kind, str)) else int(kind)
    return arr


def options(phase: int = 1, force_kind=None, validate: bool = False, inner_ratio: int = 0,
            b_transpose: Optional[L.MspCsr] = None, maskidx_max: int = -1,
            block_flops: int = -1, split_flops: int = -1, heap_flops: int = -1, kind_table=None) -> L.MspOptions:
    """msp_options; `kind_table`: see kind_table_array (the array is kept on
    the returned structure while it lives)."""
    o = L.MspOptions()
    L.load().msp_options_default(ctypes.byref(o))
    o.phase = int(phase)
    o.force_kind = KINDS[force_kind]
    o.validate = int(bool(validate))
    o.inner_ratio = int(inner_ratio)
    o.maskidx_max = int(maskidx_max)
    o.block_flops = int(block_flops)
    o.split_flops = int(split_flops)
    o.heap_flops = int(heap_flops)
    if b_transpose is not None:
        o.b_transpose = ctypes.pointer(b_transpose)
    if kind_table is not None:
        o._table = kind_table_array(kind_table)
        o.kind_table = ctypes.cast(o._table, ctypes.POINTER(ctypes.c_int8))
    return o


class Plan:
    """A plan binds the operands (row analysis + binning done once); execute
    it one or more times. The operands must stay alive and unchanged in
    pattern while the plan lives."""

    def __init__(self, A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, complement: bool = False,
                 semiring: str = "plus_times_f64", phase: int = 1, force_kind=None,
                 validate: bool = False, inner_ratio: int = 0, b_transpose: Optional[DeviceCSR] = None,
                 maskidx_max: int = -1, block_flops: int = -1, split_flops: int = -1, heap_flops: int = -1,
                 alloc=None, kind_table=None):
        """`alloc(nbytes)`: optional source of the workspaces (a uint8 device
        tensor on a 256-byte boundary, kept alive by the caller while the plan
        is used); default: torch's caching allocator. `kind_table`: a kind
        per row class (see kind_table_array)."""
        lib = L.load()
        self.semiring = semiring
        self.A, self.B, self.M = A, B, M
        self._views = (_view(A, semiring, "A"), _view(B, semiring, "B"), _view(M, None, "M"))
        self._bt = None if b_transpose is None else _view(b_transpose, semiring, "B^T")
        self._bt_keep = b_transpose
        self._opt = options(phase, force_kind, validate, inner_ratio, self._bt, maskidx_max, block_flops,
                            split_flops, heap_flops, kind_table)
        self.phase = phase
        self.nrows, self.ncols = A.nrows, B.ncols
        self.device = A.rowptr.device
        self._alloc = alloc if alloc is not None else functools.partial(_workspace, device=self.device)
        cv = int(bool(complement))
        nb = ctypes.c_size_t(0)
        _check(lib.msp_plan_workspace_size(*(ctypes.byref(v) for v in self._views), cv, SEMIRINGS[semiring],
                                           ctypes.byref(self._opt), ctypes.byref(nb)), "msp_plan_workspace_size")
        self.plan_workspace_bytes = nb.value
        self._pws = self._alloc(nb.value)
        h = ctypes.c_void_p()
        st = lib.msp_plan_create(ctypes.byref(h), *(ctypes.byref(v) for v in self._views), cv, SEMIRINGS[semiring],
                                 ctypes.byref(self._opt), ctypes.c_void_p(self._pws.data_ptr()), nb.value, _stream())
        _check(st, "msp_plan_create")
        self._h = h
        _check(lib.msp_workspace_size(self._h, ctypes.byref(nb)), "msp_workspace_size")
        self.workspace_bytes = nb.value
        self._xws = None
        info = L.MspPlanInfo()
        _check(lib.msp_plan_info(self._h, ctypes.byref(info)), "msp_plan_info")
        self.upper_bound = info.upper_bound
        self.products = info.products
        self.units = info.units
        self.staging = info.staging
        self.mask_nnz = info.mask_nnz
        self.kind_units = {k: info.kind_units[i]
                           for i, k in enumerate(["dense", "hash", "maskidx", "inner", "heap", "sort"])}
        self.bin_units = {k: info.bin_units[i] for i, k in enumerate(L.BIN_NAMES)}

    def workspace(self):
        """The execution workspace (allocated on first use, then reused)."""
        if self._xws is None:
            self._xws = self._alloc(self.workspace_bytes)
        return self._xws

    def _ws_args(self):
        ws = self.workspace()
        return ctypes.c_void_p(ws.data_ptr()), ws.numel()

    def _out(self, capacity: int, out_alloc=None):
        t = _torch()
        dev = self.A.rowptr.device
        if out_alloc is not None:
            return (_carve(out_alloc, self.nrows + 1, t.int64), _carve(out_alloc, capacity, t.int32),
                    _carve(out_alloc, capacity, out_dtype(self.semiring)))
        rp = t.empty(self.nrows + 1, dtype=t.int64, device=dev)
        ci = t.empty(max(capacity, 1), dtype=t.int32, device=dev)
        v = t.empty(max(capacity, 1), dtype=out_dtype(self.semiring), device=dev)
        return rp, ci, v

    def execute(self, nnz: bool = True, out_alloc=None) -> DeviceCSR:
        """Runs the product. Phase 1 allocates C with the upper-bound capacity
        and returns views trimmed to nnz(C) (one synchronization); phase 2
        runs symbolic, allocates exactly, then numeric. `out_alloc(nbytes)`:
        optional source of the output buffers (as `alloc` of the plan)."""
        lib = L.load()
        s = _stream()
        if self.phase == 2:
            t = _torch()
            rp = (_carve(out_alloc, self.nrows + 1, t.int64) if out_alloc is not None
                  else t.empty(self.nrows + 1, dtype=t.int64, device=self.A.rowptr.device))
            n = ctypes.c_int64(0)
            _check(lib.msp_symbolic(self._h, ctypes.c_void_p(rp.data_ptr()), ctypes.byref(n), *self._ws_args(), s),
                   "msp_symbolic")
            nn = n.value
            if out_alloc is not None:
                ci, v = _carve(out_alloc, nn, t.int32), _carve(out_alloc, nn, out_dtype(self.semiring))
            else:
                ci = t.empty(max(nn, 1), dtype=t.int32, device=rp.device)
                v = t.empty(max(nn, 1), dtype=out_dtype(self.semiring), device=rp.device)
            out = L.MspCsrOut(self.nrows, self.ncols, nn, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
            _check(lib.msp_numeric(self._h, ctypes.byref(out), *self._ws_args(), s), "msp_numeric")
            return DeviceCSR(self.nrows, self.ncols, rp, ci[:nn], v[:nn])
        rp, ci, v = self._out(self.upper_bound, out_alloc)
        out = L.MspCsrOut(self.nrows, self.ncols, self.upper_bound, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
        n = ctypes.c_int64(0)
        _check(lib.msp_execute(self._h, ctypes.byref(out), ctypes.byref(n) if nnz else None, *self._ws_args(), s),
               "msp_execute")
        if not nnz:
            return DeviceCSR(self.nrows, self.ncols, rp, ci, v)
        nn = n.value
        return DeviceCSR(self.nrows, self.ncols, rp, ci[:nn], v[:nn])

    def execute_into(self, rowptr, colidx, values, capacity: int, sync_nnz: bool = False) -> int:
        """Runs the product into caller-allocated buffers (no allocation);
        returns nnz(C) if sync_nnz, else -1 (rowptr[-1] holds it on device)."""
        lib = L.load()
        out = L.MspCsrOut(self.nrows, self.ncols, capacity, rowptr.data_ptr(), colidx.data_ptr(),
                          values.data_ptr())
        n = ctypes.c_int64(-1)
        _check(lib.msp_execute(self._h, ctypes.byref(out), ctypes.byref(n) if sync_nnz else None, *self._ws_args(),
                               _stream()), "msp_execute")
        return n.value

    def execute_profiled(self, rowptr, colidx, values, capacity: int, stage_ms) -> int:
        """Like execute_into, and adds each stage's HIP-event time (ms) to
        stage_ms (float64 numpy array of len(STAGE_NAMES)); synchronizes and
        returns nnz(C)."""
        import numpy as np
        lib = L.load()
        assert stage_ms.dtype == np.float64 and len(stage_ms) == L.NSTAGES
        out = L.MspCsrOut(self.nrows, self.ncols, capacity, rowptr.data_ptr(), colidx.data_ptr(),
                          values.data_ptr())
        n = ctypes.c_int64(-1)
        _check(lib.msp_execute_profiled(self._h, ctypes.byref(out), ctypes.byref(n), *self._ws_args(),
                                        stage_ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
               "msp_execute_profiled")
        return n.value

    def execute_timed(self, rowptr, colidx, values, capacity: int, timing: "Timing", sync_nnz: bool = False) -> int:
        """Like execute_into, recording the stage events into `timing` (read
        later by Timing.collect); returns nnz(C) if sync_nnz, else -1."""
        out = L.MspCsrOut(self.nrows, self.ncols, capacity, rowptr.data_ptr(), colidx.data_ptr(),
                          values.data_ptr())
        n = ctypes.c_int64(-1)
        _check(L.load().msp_execute_timed(self._h, ctypes.byref(out), ctypes.byref(n) if sync_nnz else None,
                                          *self._ws_args(), timing._h, _stream()), "msp_execute_timed")
        return n.value

    def row_bins(self):
        """Kernel bin of every row (numpy int8; -1 = no possible output)."""
        import numpy as np
        out = np.empty(self.nrows, dtype=np.int8)
        _check(L.load().msp_plan_row_bins(self._h, out.ctypes.data_as(ctypes.c_void_p), _stream()),
               "msp_plan_row_bins")
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.load().msp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def masked_spgemm(A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, complement: bool = False,
                  semiring: str = "plus_times_f64", phase: int = 1, force_kind=None,
                  validate: bool = False, inner_ratio: int = 0,
                  b_transpose: Optional[DeviceCSR] = None, **tuning) -> DeviceCSR:
    """C = M .* (A B) (or !M .* (A B)) over `semiring`, rows sorted.
    `tuning`: maskidx_max, block_flops, split_flops, heap_flops (binner thresholds)."""
    with Plan(A, B, M, complement, semiring, phase, force_kind, validate, inner_ratio, b_transpose,
              **tuning) as p:
        return p.execute()


def upper_bound(A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, complement: bool = False) -> int:
    lib = L.load()
    vs = (_view(A, None, "A"), _view(B, None, "B"), _view(M, None, "M"))
    nb = ctypes.c_size_t(0)
    _check(lib.msp_plan_workspace_size(*(ctypes.byref(v) for v in vs), int(bool(complement)),
                                       SEMIRINGS["plus_pair_i64"], None, ctypes.byref(nb)), "msp_plan_workspace_size")
    ws = _workspace(nb.value, A.rowptr.device)
    ub = ctypes.c_int64(0)
    _check(lib.msp_upper_bound(*(ctypes.byref(v) for v in vs), int(bool(complement)), ctypes.byref(ub),
                               ctypes.c_void_p(ws.data_ptr()), nb.value, _stream()), "msp_upper_bound")
    return ub.value


def one_shot(A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, complement: bool = False,
             semiring: str = "plus_times_f64", workspace=None, **opts):
    """msp_masked_spgemm: the one-shot product in one workspace (a uint8
    device tensor; None: sized by the call itself, which reports the bytes it
    needs). Returns (DeviceCSR, workspace bytes needed)."""
    t = _torch()
    lib = L.load()
    vs = (_view(A, semiring, "A"), _view(B, semiring, "B"), _view(M, None, "M"))
    o = options(**opts)
    dev = A.rowptr.device
    need = ctypes.c_size_t(0)
    ws = workspace
    for _ in range(3):  # at most: plan size, then whole size
        if ws is None:
            ws = _workspace(need.value, dev)
        ub = ctypes.c_int64(0)
        rp = t.empty(A.nrows + 1, dtype=t.int64, device=dev)
        # capacity from the bound: a first call with no capacity reports it
        out = L.MspCsrOut(A.nrows, B.ncols, 0, rp.data_ptr(), 0, 0)
        st = lib.msp_masked_spgemm(*(ctypes.byref(v) for v in vs), int(bool(complement)), SEMIRINGS[semiring],
                                   ctypes.byref(o), ctypes.byref(out), ctypes.byref(ub),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(need), _stream())
        if st == 5 and need.value > ws.numel():
            if workspace is not None:
                _check(st, "msp_masked_spgemm")
            ws = None
            continue
        if st == 5:  # the output capacity: ub holds the bound (phase 1) or nnz (phase 2)
            cap = max(ub.value, 1)
            ci = t.empty(cap, dtype=t.int32, device=dev)
            v = t.empty(cap, dtype=out_dtype(semiring), device=dev)
            out = L.MspCsrOut(A.nrows, B.ncols, cap, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
            n = ctypes.c_int64(0)
            _check(lib.msp_masked_spgemm(*(ctypes.byref(v_) for v_ in vs), int(bool(complement)),
                                         SEMIRINGS[semiring], ctypes.byref(o), ctypes.byref(out), ctypes.byref(n),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(need), _stream()),
                   "msp_masked_spgemm")
            return DeviceCSR(A.nrows, B.ncols, rp, ci[:n.value], v[:n.value]), need.value
        _check(st, "msp_masked_spgemm")
        return DeviceCSR(A.nrows, B.ncols, rp, t.empty(0, dtype=t.int32, device=dev),
                         t.empty(0, dtype=out_dtype(semiring), device=dev)), need.value
    raise MspError(5, "msp_masked_spgemm: workspace size did not settle")


def masked_spgemm_noalloc(A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, rowptr, colidx, values,
                          complement: bool = False, semiring: str = "plus_times_f64", **opts) -> int:
    """msp_masked_spgemm_noalloc: the one-shot product in the library's fixed
    device scratch, into caller-allocated outputs (rowptr: nrows+1 int64;
    colidx and values of equal length, the capacity). Allocates nothing;
    returns nnz(C). Raises MspError (MSP_ERR_INSUFFICIENT_CAPACITY) when the
    capacity is below the bound or the product needs more than the scratch."""
    lib = L.load()
    vs = (_view(A, semiring, "A"), _view(B, semiring, "B"), _view(M, None, "M"))
    o = options(**opts)
    cap = int(colidx.numel())
    if int(values.numel()) != cap or values.dtype != out_dtype(semiring):
        raise ValueError("values must match colidx in length and have the semiring's output type")
    out = L.MspCsrOut(A.nrows, B.ncols, cap, rowptr.data_ptr(), colidx.data_ptr() if cap else 0,
                      values.data_ptr() if cap else 0)
    n = ctypes.c_int64(0)
    need = ctypes.c_size_t(0)
    _check(lib.msp_masked_spgemm_noalloc(*(ctypes.byref(v) for v in vs), int(bool(complement)), SEMIRINGS[semiring],
                                         ctypes.byref(o), ctypes.byref(out), ctypes.byref(n), ctypes.byref(need),
                                         _stream()), "msp_masked_spgemm_noalloc")
    return n.value


class Timing:
    """A timing session: Plan.execute_timed records stage events into it
    without synchronizing; collect() waits for them and adds each stage's
    milliseconds into a float64 numpy array of len(STAGE_NAMES)."""

    def __init__(self, executions: int = 0, stages=None):
        """`executions`: create the events of that many executions now.
        `stages`: names (STAGE_NAMES) of the stages to time; None: all."""
        mask = 0
        for name in stages or ():
            mask |= 1 << L.STAGE_NAMES.index(name)
        h = ctypes.c_void_p()
        _check(L.load().msp_timing_create(ctypes.byref(h), int(executions), mask), "msp_timing_create")
        self._h = h

    def collect(self, stage_ms):
        import numpy as np
        assert stage_ms.dtype == np.float64 and len(stage_ms) == L.NSTAGES
        _check(L.load().msp_timing_collect(self._h, stage_ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "msp_timing_collect")
        return stage_ms

    def close(self):
        if getattr(self, "_h", None):
            L.load().msp_timing_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reduce_csr(rowptr, nrows: int, values, semiring: str, out=None):
    """(+)-reduction of values[:rowptr[nrows]] with the count read on the
    device (no synchronization); `values` holds at most its length."""
    t = _torch()
    if values.dtype != out_dtype(semiring):
        raise TypeError("values dtype does not match the semiring's output type")
    if out is None:
        out = t.empty(1, dtype=values.dtype, device=values.device)
    ws = _reduce_workspace(values.device)
    _check(L.load().msp_reduce_csr(ctypes.c_void_p(rowptr.data_ptr()), int(nrows),
                                   ctypes.c_void_p(values.data_ptr() if values.numel() else 0), values.numel(),
                                   SEMIRINGS[semiring], ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "msp_reduce_csr")
    return out


def _reduce_workspace(device):
    nb = ctypes.c_size_t(0)
    _check(L.load().msp_reduce_workspace_size(ctypes.byref(nb)), "msp_reduce_workspace_size")
    return _workspace(nb.value, device)


def reduce(values, semiring: str, out=None):
    """(+)-reduction of output values into a one-element device tensor."""
    t = _torch()
    if values.dtype != out_dtype(semiring):
        raise TypeError("values dtype does not match the semiring's output type")
    if out is None:
        out = t.empty(1, dtype=values.dtype, device=values.device)
    ws = _reduce_workspace(values.device)
    _check(L.load().msp_reduce(ctypes.c_void_p(values.data_ptr() if values.numel() else 0), values.numel(),
                               SEMIRINGS[semiring], ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream()), "msp_reduce")
    return out


def bc_batch(A: DeviceCSR, sources, bc=None):
    """Betweenness-centrality dependencies of a batch of sources on the
    unweighted undirected graph A (symmetric pattern, values ignored):
    adds sum over sources s != v of delta_s(v) into bc (a float64 device
    tensor of A.nrows, zeros if None). Returns (bc, info dict)."""
    import numpy as np
    t = _torch()
    src = np.ascontiguousarray(sources, dtype=np.int32)
    if bc is None:
        bc = t.zeros(A.nrows, dtype=t.float64, device=A.rowptr.device)
    view = _view(A, None, "A")
    info = L.MspBcInfo()
    mem = _TorchAllocator(A.rowptr.device)
    _check(L.load().msp_bc_batch(ctypes.byref(view), ctypes.c_void_p(src.ctypes.data if len(src) else 0),
                                 len(src), ctypes.c_void_p(bc.data_ptr() if bc.numel() else 0),
                                 ctypes.byref(info), ctypes.byref(mem.struct), _stream()), "msp_bc_batch")
    res = {f: getattr(info, f) for f, _ in L.MspBcInfo._fields_}
    res["peak_device_bytes"] = mem.peak
    return bc, res


def ktruss(A: DeviceCSR, k: int):
    """k-truss of the undirected graph A (symmetric pattern): the edges with
    at least k - 2 triangles inside the truss, by repeated masked products.
    Returns (DeviceCSR of the truss with int64 supports as values, info)."""
    t = _torch()
    dev = A.rowptr.device
    rp = t.empty(A.nrows + 1, dtype=t.int64, device=dev)
    cap = max(A.colidx.numel(), 1)
    ci = t.empty(cap, dtype=t.int32, device=dev)
    sup = t.empty(cap, dtype=t.int64, device=dev)
    view = _view(A, None, "A")
    n = ctypes.c_int64(0)
    info = L.MspKtrussInfo()
    mem = _TorchAllocator(dev)
    _check(L.load().msp_ktruss(ctypes.byref(view), int(k), ctypes.c_void_p(rp.data_ptr()),
                               ctypes.c_void_p(ci.data_ptr()), ctypes.c_void_p(sup.data_ptr()), ctypes.byref(n),
                               ctypes.byref(info), ctypes.byref(mem.struct), _stream()), "msp_ktruss")
    nn = n.value
    res = {f: getattr(info, f) for f, _ in L.MspKtrussInfo._fields_}
    res["peak_device_bytes"] = mem.peak
    return DeviceCSR(A.nrows, A.ncols, rp, ci[:nn], sup[:nn]), res


def version() -> int:
    return L.load().msp_version()


class Batch:
    """Many masked products on one semiring planned and run together: each
    kernel bin is one launch over the units of every product; execute() can
    be captured once into a HIP graph and replayed (graph_launch()).

    problems: list of (A, B, M, complement) DeviceCSR triples."""

    def __init__(self, problems, semiring: str = "plus_times_f64", force_kind=None, inner_ratio: int = 0,
                 maskidx_max: int = -1, block_flops: int = -1, split_flops: int = -1, heap_flops: int = -1,
                 alloc=None, kind_table=None):
        """`alloc(nbytes)`: optional source of the workspaces (as for Plan);
        `kind_table`: a kind per row class (see kind_table_array)."""
        lib = L.load()
        self.semiring = semiring
        self.problems = list(problems)
        n = len(self.problems)
        arr = (L.MspProblem * n)()
        for p, (A, B, M, comp) in enumerate(self.problems):
            arr[p].A = _view(A, semiring, "A")
            arr[p].B = _view(B, semiring, "B")
            arr[p].M = _view(M, None, "M")
            arr[p].complement = int(bool(comp))
        self._arr = arr
        self._opt = options(1, force_kind, False, inner_ratio, None, maskidx_max, block_flops, split_flops,
                            heap_flops, kind_table)
        self.device = self.problems[0][0].rowptr.device if n else None
        nb = ctypes.c_size_t(0)
        _check(lib.msp_batch_workspace_size(arr, n, SEMIRINGS[semiring], ctypes.byref(self._opt), ctypes.byref(nb)),
               "msp_batch_workspace_size")
        self.plan_workspace_bytes = nb.value
        self._alloc = alloc if alloc is not None else functools.partial(_workspace, device=self.device)
        self._pws = self._alloc(nb.value)
        h = ctypes.c_void_p()
        _check(lib.msp_batch_create(ctypes.byref(h), arr, n, SEMIRINGS[semiring], ctypes.byref(self._opt),
                                    ctypes.c_void_p(self._pws.data_ptr()), nb.value, _stream()), "msp_batch_create")
        self._h = h
        _check(lib.msp_workspace_size(self._h, ctypes.byref(nb)), "msp_workspace_size")
        self.workspace_bytes = nb.value
        self._xws = None
        self.count = n
        self.upper_bounds = []
        self.products = []
        for p in range(n):
            info = L.MspPlanInfo()
            _check(lib.msp_batch_info(h, p, ctypes.byref(info)), "msp_batch_info")
            self.upper_bounds.append(info.upper_bound)
            self.products.append(info.products)
        info = L.MspPlanInfo()
        _check(lib.msp_batch_info(h, -1, ctypes.byref(info)), "msp_batch_info")
        self.units = info.units
        self.bin_units = {k: info.bin_units[i] for i, k in enumerate(L.BIN_NAMES)}
        self.outputs = None

    def bind_new_outputs(self, out_alloc=None, keep=None):
        """Allocates every output with its upper-bound capacity and binds it.
        `out_alloc(nbytes)`: optional source of the output buffers, except
        for the products p with keep[p] true, which get their own. By default
        all outputs are views into one device allocation (one allocation
        instead of three per product; a kept result keeps that allocation
        alive)."""
        t = _torch()
        outs = (L.MspCsrOut * self.count)()
        self.outputs = []
        if out_alloc is None and self.count:
            w = t.empty(0, dtype=out_dtype(self.semiring)).element_size()
            total = sum(_Slab.size((A.nrows + 1) * 8) + _Slab.size(max(self.upper_bounds[p], 1) * 4) +
                        _Slab.size(max(self.upper_bounds[p], 1) * w)
                        for p, (A, _, _, _) in enumerate(self.problems))
            out_alloc, keep = _Slab(total, self.problems[0][0].rowptr.device), None
        for p, (A, B, M, _) in enumerate(self.problems):
            dev = A.rowptr.device
            cap = max(self.upper_bounds[p], 1)
            if out_alloc is not None and not (keep is not None and keep[p]):
                rp, ci, v = (_carve(out_alloc, A.nrows + 1, t.int64), _carve(out_alloc, cap, t.int32),
                             _carve(out_alloc, cap, out_dtype(self.semiring)))
            else:
                rp = t.empty(A.nrows + 1, dtype=t.int64, device=dev)
                ci = t.empty(cap, dtype=t.int32, device=dev)
                v = t.empty(cap, dtype=out_dtype(self.semiring), device=dev)
            self.outputs.append((rp, ci, v))
            outs[p] = L.MspCsrOut(A.nrows, B.ncols, cap, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
        if self._xws is None:
            self._xws = self._alloc(self.workspace_bytes)
        _check(L.load().msp_batch_bind(self._h, outs, ctypes.c_void_p(self._xws.data_ptr()), self._xws.numel(),
                                       _stream()), "msp_batch_bind")
        return self.outputs

    def execute(self):
        _check(L.load().msp_batch_execute(self._h, _stream()), "msp_batch_execute")

    def execute_timed(self, timing: "Timing"):
        """execute() with the stage events recorded into `timing`."""
        _check(L.load().msp_batch_execute_timed(self._h, timing._h, _stream()), "msp_batch_execute_timed")

    def row_bins(self):
        """Kernel bin of every row of every product, products one after
        another (numpy int8; -1 = no possible output)."""
        import numpy as np
        out = np.empty(sum(A.nrows for (A, _, _, _) in self.problems), dtype=np.int8)
        _check(L.load().msp_plan_row_bins(self._h, out.ctypes.data_as(ctypes.c_void_p), _stream()),
               "msp_plan_row_bins")
        return out

    def graph_launch(self):
        """Replays the captured graph (captures it on first use); the current
        stream must not be the default stream."""
        _check(L.load().msp_batch_graph_launch(self._h, _stream()), "msp_batch_graph_launch")

    def results(self):
        """Outputs trimmed to nnz (synchronizes)."""
        n = (ctypes.c_int64 * self.count)()
        _check(L.load().msp_batch_nnz(self._h, n, _stream()), "msp_batch_nnz")
        res = []
        for p, (rp, ci, v) in enumerate(self.outputs):
            A, B = self.problems[p][0], self.problems[p][1]
            res.append(DeviceCSR(A.nrows, B.ncols, rp, ci[:n[p]], v[:n[p]]))
        return res

    def close(self):
        if getattr(self, "_h", None):
            L.load().msp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
