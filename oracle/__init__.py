"""CPU oracle for C = M .* (A B) over a semiring (plain C, OpenMP over rows).

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports, links or calls it, and the two share no code.

The arithmetic lives in ``msp_oracle.c`` (Algorithm 1 row-wise Gustavson
product, then the mask filter on the mask pattern, then ascending column
order). This wrapper only marshals numpy arrays through ctypes.

Operands are duck-typed CSR objects with attributes ``nrows``, ``ncols``,
``rowptr`` (int64), ``colidx`` (int32) and ``values`` (array or None).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msp_oracle.c")
_SRC_BC = os.path.join(_HERE, "bc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SEMIRINGS = {
    "plus_times_f64": 0,
    "plus_pair_i64": 1,
    "lor_land_bool": 2,
    "plus_times_i32": 3,
    "plus_times_i64": 4,
}
IN_DTYPE = {0: np.float64, 1: None, 2: np.uint8, 3: np.int32, 4: np.int64}
OUT_DTYPE = {0: np.float64, 1: np.int64, 2: np.uint8, 3: np.int32, 4: np.int64}


class _Result(ctypes.Structure):
    _fields_ = [
        ("nrows", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("rowptr", ctypes.POINTER(ctypes.c_int64)),
        ("colidx", ctypes.POINTER(ctypes.c_int32)),
        ("values", ctypes.c_void_p),
        ("useful", ctypes.POINTER(ctypes.c_int64)),
    ]


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", _SRC, _SRC_BC, "-o", _LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.oracle_masked_spgemm.restype = ctypes.POINTER(_Result)
        lib.oracle_masked_spgemm.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            vp, vp, vp, vp, vp, vp, vp, vp,
            ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_bc.restype = ctypes.c_int
        lib.oracle_bc.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _vals(X, sr):
    dt = IN_DTYPE[sr]
    if dt is None or X.values is None:
        return None
    return np.ascontiguousarray(X.values, dtype=dt)


class Result:
    """Rows of C as numpy CSR (rowptr over the computed rows) plus the number
    of admitted products per computed row."""

    def __init__(self, nrows, ncols, rowptr, colidx, values, useful, rows):
        self.nrows, self.ncols = nrows, ncols
        self.rowptr, self.colidx, self.values = rowptr, colidx, values
        self.useful = useful
        self.rows = rows

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def masked_spgemm(A, B, M, complement: bool = False, semiring: str = "plus_times_f64",
                  rows: Optional[np.ndarray] = None, nthreads: int = 0) -> Result:
    """C = M .* (A B) (or !M .* (A B) with ``complement``) on the CPU.

    ``rows`` selects a subset of rows (in the given order, repeats allowed);
    the result then holds only those rows. ``nthreads`` = 0 uses OpenMP's
    default thread count."""
    sr = SEMIRINGS[semiring]
    if A.ncols != B.nrows or M.nrows != A.nrows or M.ncols != B.ncols:
        raise ValueError("dimension mismatch")
    lib = _load()
    Arp = np.ascontiguousarray(A.rowptr, np.int64)
    Aci = np.ascontiguousarray(A.colidx, np.int32)
    Brp = np.ascontiguousarray(B.rowptr, np.int64)
    Bci = np.ascontiguousarray(B.colidx, np.int32)
    Mrp = np.ascontiguousarray(M.rowptr, np.int64)
    Mci = np.ascontiguousarray(M.colidx, np.int32)
    Av, Bv = _vals(A, sr), _vals(B, sr)
    sel = None if rows is None else np.ascontiguousarray(rows, np.int64)
    nsel = A.nrows if sel is None else len(sel)
    r = lib.oracle_masked_spgemm(A.nrows, A.ncols, B.ncols,
                                 _ptr(Arp), _ptr(Aci), _ptr(Av),
                                 _ptr(Brp), _ptr(Bci), _ptr(Bv),
                                 _ptr(Mrp), _ptr(Mci),
                                 int(bool(complement)), sr, _ptr(sel), nsel, int(nthreads))
    if not r:
        raise MemoryError("oracle failed")
    try:
        res = r.contents
        nr, nnz = res.nrows, res.nnz
        rowptr = np.ctypeslib.as_array(res.rowptr, shape=(nr + 1,)).copy()
        colidx = (np.ctypeslib.as_array(res.colidx, shape=(nnz,)).copy()
                  if nnz else np.zeros(0, np.int32))
        odt = OUT_DTYPE[sr]
        if nnz:
            buf = (ctypes.c_char * (nnz * np.dtype(odt).itemsize)).from_address(res.values)
            values = np.frombuffer(buf, dtype=odt).copy()
        else:
            values = np.zeros(0, odt)
        useful = (np.ctypeslib.as_array(res.useful, shape=(nr,)).copy()
                  if nr else np.zeros(0, np.int64))
    finally:
        lib.oracle_free(r)
    return Result(nsel, B.ncols, rowptr, colidx, values, useful, sel)


def bc(G, sources, nthreads: int = 0) -> np.ndarray:
    """Betweenness-centrality dependencies of a batch of sources on the
    unweighted undirected graph G (symmetric CSR pattern): bc[v] = sum over
    the sources s != v of delta_s(v) (Brandes; see bc_oracle.c)."""
    lib = _load()
    if G.nrows != G.ncols:
        raise ValueError("G must be square")
    rp = np.ascontiguousarray(G.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(G.colidx, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(G.nrows, dtype=np.float64)
    st = lib.oracle_bc(G.nrows, rp.ctypes.data, ci.ctypes.data, len(src), src.ctypes.data, out.ctypes.data,
                       int(nthreads))
    if st != 0:
        raise ValueError("oracle_bc failed (bad source or out of memory)")
    return out


def ktruss(G, k: int):
    """k-truss of the undirected graph G (symmetric pattern) by the paper's
    iteration (Section "Experimental Setup"): repeat S = C .* (C C) under
    plus-pair with the oracle's masked product, keep the entries with
    support >= k - 2, until no edge is removed. k <= 2 returns G with
    supports 0. Returns (rowptr, colidx, support) as numpy arrays."""
    n = G.nrows
    rp = np.asarray(G.rowptr, dtype=np.int64)
    ci = np.asarray(G.colidx, dtype=np.int32)
    if k <= 2 or len(ci) == 0:
        return rp.copy(), ci.copy(), np.zeros(len(ci), dtype=np.int64)

    class _C:  # duck-typed CSR for masked_spgemm
        def __init__(self, rp, ci):
            self.nrows, self.ncols, self.rowptr, self.colidx, self.values = n, n, rp, ci, None

    sup = np.zeros(len(ci), dtype=np.int64)
    while True:
        C = _C(rp, ci)
        S = masked_spgemm(C, C, C, False, "plus_pair_i64")
        keep = S.values >= k - 2
        rows = np.repeat(np.arange(n), np.diff(S.rowptr))[keep]
        nrp = np.zeros(n + 1, dtype=np.int64)
        np.add.at(nrp, rows + 1, 1)
        nrp = np.cumsum(nrp)
        nci = S.colidx[keep].astype(np.int32)
        sup = S.values[keep].astype(np.int64)
        done = len(nci) == len(ci)
        rp, ci = nrp, nci
        if done or len(ci) == 0:
            return rp, ci, sup
