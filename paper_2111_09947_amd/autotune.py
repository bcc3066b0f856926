"""Autotuner for the row binner: picks, for a given set of products, the
binner thresholds that run fastest, keeping the outputs unchanged.

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
