"""CPU-baseline leg of the benchmark: times the oracle on operands that the
benchmark saved to a directory, in a process of its own.

TEST INFRASTRUCTURE ONLY, like the rest of this package. It runs as a child
process (``python -m oracle.bench_leg DIR``) so that the OpenMP thread
binding it asks for (OMP_PROC_BIND=close, set by the parent in the child's
environment) pins only the oracle's threads and none of the benchmark's.

DIR holds ``spec.json`` and the operands as ``.npy`` files:
  spec: {"complement": bool, "semiring": str, "reps": int,
         "threads": [thread counts to try], "one_thread_rows": bool,
         "sample": bool}
  A_rowptr, A_colidx, [A_values], B_..., M_rowptr, M_colidx, shape.npy
  (m, k, n), and optionally rows.npy (the rows of the timed sample) and
  rows_one.npy (the rows of the one-thread run).
It prints one JSON line: per thread count the run times, and the admitted
products (the useful-flop numerator) of the sample; with "sample" it also
saves the sample's result rows (C_rowptr, C_colidx, C_values) into DIR for
the parent's parity check.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from oracle import masked_spgemm


class _CSR:
    def __init__(self, nrows, ncols, rowptr, colidx, values):
        self.nrows, self.ncols = nrows, ncols
        self.rowptr, self.colidx, self.values = rowptr, colidx, values


def _load(d, name, nrows, ncols):
    def get(part):
        p = os.path.join(d, f"{name}_{part}.npy")
        return np.load(p) if os.path.exists(p) else None
    return _CSR(nrows, ncols, get("rowptr"), get("colidx"), get("values"))


def main(d: str) -> None:
    with open(os.path.join(d, "spec.json")) as fh:
        spec = json.load(fh)
    m, k, n = (int(x) for x in np.load(os.path.join(d, "shape.npy")))
    A = _load(d, "A", m, k)
    B = _load(d, "B", k, n)
    M = _load(d, "M", m, n)
    rows_p = os.path.join(d, "rows.npy")
    rows = np.load(rows_p) if os.path.exists(rows_p) else None
    comp, sr, reps = bool(spec["complement"]), spec["semiring"], int(spec["reps"])
    out = {"runs": {}}
    R = None
    for nt in spec["threads"]:
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            R = masked_spgemm(A, B, M, comp, sr, rows=rows, nthreads=int(nt))
            times.append(time.perf_counter() - t0)
        out["runs"][str(nt)] = times
    out["useful"] = int(R.useful.sum())
    out["nnz"] = int(R.nnz)
    if sr in ("plus_pair_i64", "plus_times_i64", "plus_times_i32"):
        out["sum"] = int(R.values.astype(np.int64).sum())
    if spec.get("sample"):
        np.save(os.path.join(d, "C_rowptr.npy"), R.rowptr)
        np.save(os.path.join(d, "C_colidx.npy"), R.colidx)
        np.save(os.path.join(d, "C_values.npy"), R.values)
    del R
    one_p = os.path.join(d, "rows_one.npy")
    if spec.get("one_thread_rows") and os.path.exists(one_p):
        rows1 = np.load(one_p)
        t0 = time.perf_counter()
        R1 = masked_spgemm(A, B, M, comp, sr, rows=rows1, nthreads=1)
        out["one_thread"] = {"seconds": time.perf_counter() - t0, "useful": int(R1.useful.sum()),
                             "rows": int(len(rows1))}
    elif spec.get("one_thread_rows"):
        t0 = time.perf_counter()
        R1 = masked_spgemm(A, B, M, comp, sr, rows=rows, nthreads=1)
        out["one_thread"] = {"seconds": time.perf_counter() - t0, "useful": int(R1.useful.sum()),
                             "rows": int(m if rows is None else len(rows))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
