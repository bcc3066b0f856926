"""Autotuners for the row binner, keeping the outputs unchanged:

- autotune_classes picks the accumulator kind per row class (the bucket of
  the row's product count x the bucket of its mask row length, the classes
  of msp_options.kind_table) for a given batch of products, class by class
  from the heaviest, timing the whole batch for every candidate kind;
- autotune searches global binner thresholds over a small grid.

The tunables decide which accumulator kind and work-group shape a row class
gets (they are plan options of the C-ABI):
  maskidx_max  rows whose mask has at most this many entries use the
               binary-search (mask-indexed) kind, larger ones the hash kind
  block_flops  rows with more products than this run on a 256-thread
               work-group instead of a single wavefront
  inner_ratio  0, or use the pull (inner-product) kind for rows whose pull
               cost times this ratio is below their push cost

Every candidate's outputs are compared with the first candidate's: patterns
exactly, integer values exactly, FP64 values within 1e-12 relative. A
candidate that changes an output is rejected (raises).
"""
from __future__ import annotations

import gc
import itertools
import json
import time
from typing import Dict, List, Optional

DEFAULT_SPACE = {
    "maskidx_max": [0, 8, 32],
    "block_flops": [2048, 8192, 32768],
    "inner_ratio": [0],
}

FP64_RTOL = 1e-12


def same_output(rowptr, colidx, values, ref_rowptr, ref_colidx, ref_values, fp64: bool) -> bool:
    """Patterns exactly; values exactly, or within 1e-12 relative for FP64."""
    import torch
    if not (torch.equal(rowptr, ref_rowptr) and torch.equal(colidx, ref_colidx)):
        return False
    if fp64:
        d = (values - ref_values).abs()
        return bool((d <= FP64_RTOL * ref_values.abs()).all().item())
    return torch.equal(values, ref_values)


def autotune(problems, semiring: str, space: Optional[Dict[str, List[int]]] = None, repeats: int = 3,
             use_graph: bool = True, out_path: Optional[str] = None) -> dict:
    """problems: list of (A, B, M, complement) DeviceCSR tuples (one batch).
    Times each configuration of `space` over `repeats` batched executions
    (graph replays when use_graph) and returns
    {"best": {...}, "trials": [{"config":..., "ms":...}, ...]}."""
    import torch

    from . import Batch

    space = dict(DEFAULT_SPACE if space is None else space)
    keys = sorted(space)
    reference = None
    trials = []
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for values in itertools.product(*(space[k] for k in keys)):
            cfg = dict(zip(keys, values))
            with Batch(problems, semiring=semiring, **cfg) as b:
                b.bind_new_outputs()
                run = b.graph_launch if use_graph else b.execute
                run()  # warm-up (and capture)
                stream.synchronize()
                t0 = time.perf_counter()
                for _ in range(repeats):
                    run()
                stream.synchronize()
                ms = (time.perf_counter() - t0) / repeats * 1e3
                res = b.results()
                if reference is None:
                    reference = [(r.rowptr.clone(), r.colidx.clone(), r.values.clone()) for r in res]
                else:
                    for r, (rp, ci, v) in zip(res, reference):
                        if not same_output(r.rowptr, r.colidx, r.values, rp, ci, v, semiring == "plus_times_f64"):
                            raise RuntimeError(f"configuration {cfg} changed an output")
                trials.append({"config": cfg, "ms": round(ms, 4)})
    best = min(trials, key=lambda t: t["ms"])
    result = {"semiring": semiring, "best": best["config"], "best_ms": best["ms"], "trials": trials}
    if out_path:
        with open(out_path, "w") as f:
            json.dump(result, f, indent=1)
    return result


KIND_NAMES = ("dense", "hash", "maskidx", "inner", "heap")


def _bucket(x):
    """Bucket b of a count: 4^b <= x < 4^(b+1), 0 below 4, the last one above."""
    import torch
    from . import _lib as L
    b = torch.floor(torch.log2(x.clamp(min=1).double()) / 2).long()
    return b.clamp(0, L.ROW_BUCKETS - 1)


def row_classes(problems):
    """(class index per row, products per row) of every product's rows, on
    the device: class = bucket(products) * ROW_BUCKETS + bucket(mask row
    length), products = sum over A(i,:) of nnz(B(k,:))."""
    import torch
    from . import _lib as L
    cls, work = [], []
    for (A, B, M, _c) in problems:
        bdeg = (B.rowptr[1:] - B.rowptr[:-1])
        adeg = (A.rowptr[1:] - A.rowptr[:-1])
        per = bdeg[A.colidx.long()] if A.colidx.numel() else torch.zeros(0, dtype=torch.int64, device=A.rowptr.device)
        cs = torch.cumsum(torch.cat([torch.zeros(1, dtype=torch.int64, device=per.device), per]), 0)
        fl = cs[A.rowptr[1:]] - cs[A.rowptr[:-1]]
        mn = M.rowptr[1:] - M.rowptr[:-1]
        cls.append(_bucket(fl) * L.ROW_BUCKETS + _bucket(mn))
        work.append(fl)
        del adeg
    return torch.cat(cls), torch.cat(work)


def autotune_classes(problems, semiring: str, kinds=KIND_NAMES, min_share: float = 0.02, repeats: int = 3,
                     gain: float = 0.02, out_path: Optional[str] = None) -> dict:
    """Kind per row class for one batch. The classes holding at least
    `min_share` of all products are tuned one after another, heaviest
    first: each candidate kind is timed on the whole batch (graph replays,
    median of `repeats`, the table so far plus the candidate), and it is kept
    when it beats the best so far by more than `gain`. A candidate more than
    three times slower than the best is dropped after one run. Every output
    is compared with the untuned one (patterns exactly, values exactly or
    within 1e-12 relative for FP64); a candidate that changes one raises.
    Returns {"table": {class: kind}, "default_ms", "best_ms", "trials": [...]}."""
    import torch

    from . import Batch
    from . import _lib as L

    cls, work = row_classes(problems)
    total = float(work.sum().item()) or 1.0
    per_class = torch.bincount(cls, weights=work.double(), minlength=L.KIND_CLASSES).cpu().numpy()
    order = [int(c) for c in per_class.argsort()[::-1] if per_class[c] / total >= min_share]
    stream = torch.cuda.Stream()
    reference = None
    trials = []

    ws_limit = None

    def run(table):
        """Median replay time of the batch under `table`, or None when its
        execution workspace exceeds ws_limit (a kind whose tiles multiply
        the staging) or the device runs out of memory."""
        nonlocal reference
        gc.collect()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            with Batch(problems, semiring=semiring, kind_table=table or None) as b:
                if ws_limit is not None and b.workspace_bytes > ws_limit:
                    return None
                try:
                    b.bind_new_outputs()
                except torch.OutOfMemoryError:
                    b.outputs = None
                    torch.cuda.empty_cache()
                    return None
                b.graph_launch()  # capture and first replay
                stream.synchronize()
                times = []
                for r in range(repeats):
                    t0 = time.perf_counter()
                    b.graph_launch()
                    stream.synchronize()
                    times.append((time.perf_counter() - t0) * 1e3)
                    if r == 0 and best_ms is not None and times[0] > 3 * best_ms:
                        break
                res = b.results()
                if reference is None:
                    reference = [(x.rowptr.clone(), x.colidx.clone(), x.values.clone()) for x in res]
                else:
                    for x, (rp, ci, v) in zip(res, reference):
                        if not same_output(x.rowptr, x.colidx, x.values, rp, ci, v, semiring == "plus_times_f64"):
                            raise RuntimeError(f"kind table {table} changed an output")
        return float(sorted(times)[len(times) // 2])

    best_ms = None
    default_ms = run({})
    best_ms = default_ms
    with Batch(problems, semiring=semiring) as b0:  # candidates may use up to twice its workspace
        ws_limit = 2 * b0.workspace_bytes
    table = {}
    for c in order:
        key = (c // L.ROW_BUCKETS, c % L.ROW_BUCKETS)
        for kind in kinds:
            cand = dict(table)
            cand[key] = kind
            ms = run(cand)
            trials.append({"class": list(key), "share": round(float(per_class[c] / total), 4), "kind": kind,
                           "ms": None if ms is None else round(ms, 4)})
            if ms is not None and ms < best_ms * (1 - gain):
                best_ms, table = ms, cand
    gc.collect()
    torch.cuda.empty_cache()
    result = {"semiring": semiring, "table": {f"{k[0]},{k[1]}": v for k, v in table.items()},
              "default_ms": round(default_ms, 4), "best_ms": round(best_ms, 4), "trials": trials}
    if out_path:
        with open(out_path, "w") as f:
            json.dump(result, f, indent=1)
    return result


def table_from_result(result):
    """The kind table of an autotune_classes result, for Plan / Batch."""
    return {tuple(int(x) for x in k.split(",")): v for k, v in result["table"].items()}
