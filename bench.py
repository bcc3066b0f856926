#!/usr/bin/env python3
"""Benchmark of the masked SpGEMM hot path on one MI355X.

Default run (one JSON line), three workloads, each timed as whole steps on
device-resident operands (row analysis and binning, i.e. plan creation, the
one-phase numeric kernels into staging, prefix sum of the counts, row
pointers, compaction into C, and any post-reduction):

  - headline: one multi-source BFS step, C = !V .* (A F), on an R-MAT graph
    of scale 20, edge factor 16 (Graph500 quadrant probabilities .57, .19,
    .19, symmetrized), 512 sources at depths 1..3, complemented visited mask,
    int32 path counts (the boolean semiring as a second record);
  - triangle counting on R-MAT scale 18, edge factor 16, degree-relabelled:
    C = L .* (L L) under plus-pair (int64), then the sum of C (Section
    "Triangle Counting");
  - Erdos-Renyi A, B, M with n = 4096 and average degree 8, FP64 plus-times,
    normal mask.

Inputs are synthetic and seeded; they stand in for the paper's inputs. For
each workload the line holds the useful masked GFLOP/s (2 x admitted
products / step time), the HBM roofline of the dominant numeric kernel
(algorithmic bytes of the push method per launch / its HIP-event time), the
whole step's fraction of the HBM peak under the same byte model, an oracle
check of the result, and the CPU oracle's rate on a stated sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# serving: requests with more products than this run alone (never grouped)
GROUP_WORK_MAX = 20_000_000


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("msp_kernels.hip", "msp_device.hpp", "msp_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2111_09947_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tuning_kw(args):
    """Binner thresholds given on the command line (0 keeps the library's)."""
    kw = {}
    for name in ("maskidx_max", "block_flops", "split_flops"):
        v = getattr(args, name, 0)
        if v:
            kw[name] = v
    if getattr(args, "heap_flops", None) is not None:
        kw["heap_flops"] = args.heap_flops
    return kw


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_info(dev):
    """The properties of the GPU the run used (as the runtime reports them)."""
    import torch
    p = torch.cuda.get_device_properties(dev)
    keys = ("name", "gcnArchName", "multi_processor_count", "total_memory", "L2_cache_size",
            "shared_memory_per_block", "max_threads_per_multi_processor", "regs_per_multiprocessor", "warp_size")
    return {k: getattr(p, k) for k in keys if hasattr(p, k)}


def other_stages(make_plan, nrows, dtype, stage_ms, steps, dev, runs=2, keep=None):
    """Times the stages other than the kernel bins (scans, row pointers,
    compaction, split emission), and the bins other than `keep` (the stage
    timed live), in `runs` untimed profiled executions and stores them in
    stage_ms scaled to `steps` steps."""
    import torch

    import paper_2111_09947_amd as msp
    extra = np.zeros_like(stage_ms)
    for _ in range(runs):
        with make_plan() as p:
            cap = max(p.upper_bound, 1)
            p.execute_profiled(torch.empty(nrows + 1, dtype=torch.int64, device=dev),
                               torch.empty(cap, dtype=torch.int32, device=dev),
                               torch.empty(cap, dtype=dtype, device=dev), cap, extra)
    if keep is None:
        nb = len(msp.BIN_NAMES)
        stage_ms[nb:] = extra[nb:] / runs * steps
    else:
        for x in range(len(stage_ms)):
            if x != keep:
                stage_ms[x] = extra[x] / runs * steps


def row_quantities(L):
    """Per-row counts of the push method for A = B = M = L: A row length,
    products flops_i = sum over k in row i of nnz(L(k,:)), mask length."""
    deg = np.diff(L.rowptr)
    rows = np.repeat(np.arange(L.nrows), deg)
    flops = np.bincount(rows, weights=deg[L.colidx], minlength=L.nrows).astype(np.int64)
    return deg.astype(np.int64), flops, deg.astype(np.int64)


def alg_bytes(nnzA, flops, mnnz, useful, nnzC, wA=0, wB=0, wC=8):
    """Algorithmic bytes of the row-wise push method (memory traffic model of
    Section "Push-Based algorithms": A rows, B row pointers, B stanzas, B
    values of admitted products only, mask pattern, C write), per row."""
    return (8 + nnzA * (4 + wA)          # A row pointer and row
            + 16 * nnzA                  # B row pointer pair per A entry
            + 4 * flops                  # B column indices of every product
            + wB * useful                # B values of admitted products
            + 8 + 4 * mnnz               # mask row pointer and pattern
            + 8 + nnzC * (4 + wC))       # output count / row pointer and entries


def load_traffic(path, kernel_hash, bin_name):
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash or t.get("bin") != bin_name:
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=18)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=18)
    ap.add_argument("--phase", type=int, default=1, choices=(1, 2))
    ap.add_argument("--force-kind", default=None, choices=(None, "dense", "hash", "maskidx", "inner"))
    ap.add_argument("--inner-ratio", type=int, default=0)
    ap.add_argument("--maskidx-max", type=int, default=0, help="binner: mask rows up to this length use the "
                    "search kind (0: library default)")
    ap.add_argument("--block-flops", type=int, default=0, help="binner: products per row above which a row "
                    "takes a workgroup (0: library default)")
    ap.add_argument("--split-flops", type=int, default=0, help="binner: products per row above which a dense "
                    "row is split over workgroups (0: library default)")
    ap.add_argument("--heap-flops", type=int, default=None, help="binner: rows with at most this many products "
                    "(and at most 8 entries in A's row) use the heap kind (0: never; default: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="all",
                    choices=("all", "tc", "er", "er_batch", "batch", "bfs", "complement", "serve", "bc", "ktruss",
                             "heatmap", "copy"),
                    help="all (default): the multi-source BFS step (headline), triangle counting and the "
                         "Erdos-Renyi n=4096 product in one line; tc, er, bfs: one of them; er_batch: 256 "
                         "Erdos-Renyi n=4096 products as one batch; batch: 64 mixed FP64 "
                         "products, batched and graph-replayed vs one launch per product; complement: "
                         "an Erdos-Renyi product over 2^20 columns under a complemented mask")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--mask-cap", type=int, default=0,
                    help="batch: cap on one product's mask entries (0: none, the full-size masks)")
    ap.add_argument("--no-tune", action="store_true", help="batch: skip tuning the accumulator kind per row class")
    ap.add_argument("--requests", type=int, default=2000, help="serve: measured requests")
    ap.add_argument("--slots", type=int, default=4, help="serve: concurrent execution slots")
    ap.add_argument("--summarize-traffic", metavar="DIR", default=None,
                    help="turn the FETCH_SIZE / WRITE_SIZE counter runs under DIR (copy_FETCH_SIZE, copy_WRITE_SIZE, "
                         "KEY_FETCH_SIZE, KEY_WRITE_SIZE) into profiles/traffic_KEY.json for --bin/--kernel")
    ap.add_argument("--traffic-key", default="tc_rmat18", help="with --summarize-traffic: the workload key "
                    "(tc_rmat18, bfs_rmat20_i32, bfs_rmat20_bool, er4096, er4096_x256)")
    ap.add_argument("--bin", default="hash_block", help="with --summarize-traffic: the kernel bin")
    ap.add_argument("--kernel", default="k_maskkey<1, 1, 4, 512, true, 1, false>",
                    help="with --summarize-traffic: the kernel name (substring) of that bin")
    args = ap.parse_args()

    if args.summarize_traffic:
        return summarize_traffic(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build "
              "(the row-sharded multi-GPU design is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "bfs":
        return run_bfs(args)
    if args.workload == "bc":
        return run_bc(args)
    if args.workload == "ktruss":
        return run_ktruss(args)
    if args.workload == "heatmap":
        return run_heatmap(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "copy":
        return run_copy(args)
    if args.workload == "tc":
        return run_tc(args)
    if args.workload == "er":
        return run_er(args)
    if args.workload == "complement":
        return print(json.dumps(headline(measure_complement(args), args)), flush=True)
    if args.workload == "er_batch":
        return print(json.dumps(headline(measure_er_batched(args), args)), flush=True)
    run_all(args)


# ----------------------------------------------------------------------------------------------
# measurement core: one product timed as whole steps (plan creation included), its stages, the
# byte model per row, the dominant kernel's roofline, and the oracle's CPU leg


def sig(x, digits=5):
    """x rounded to `digits` significant digits."""
    return float(f"{x:.{digits}g}")


def cpu_threads():
    """(host cores this process may run on, the cgroup's CPU quota in cores
    or None when unlimited)."""
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()[:2]
        if q != "max":
            quota = max(1, int(-(-int(q) // int(per))))
    except (OSError, ValueError):
        pass
    return aff, quota


def cpu_leg(A, B, M, complement, sr, rows=None, rows_one=None, reps=5, sample=False):
    """Runs the oracle in a child process (oracle/bench_leg.py) on these host
    operands with every host core the process may use (and the cgroup quota,
    when it is lower), threads bound close (OMP_PROC_BIND=close). Returns
    the child's report plus, with `sample`, the oracle's result rows."""
    import shutil
    import subprocess
    import tempfile
    d = tempfile.mkdtemp(prefix="msp_cpu_leg_", dir="/tmp")
    try:
        np.save(os.path.join(d, "shape.npy"), np.array([A.nrows, A.ncols, B.ncols], np.int64))
        for name, X in (("A", A), ("B", B), ("M", M)):
            np.save(os.path.join(d, f"{name}_rowptr.npy"), X.rowptr)
            np.save(os.path.join(d, f"{name}_colidx.npy"), X.colidx)
            if X.values is not None and name != "M":
                np.save(os.path.join(d, f"{name}_values.npy"), X.values)
        if rows is not None:
            np.save(os.path.join(d, "rows.npy"), np.asarray(rows, np.int64))
        if rows_one is not None:
            np.save(os.path.join(d, "rows_one.npy"), np.asarray(rows_one, np.int64))
        aff, quota = cpu_threads()
        threads = [aff] + ([quota] if quota is not None and quota < aff else [])
        with open(os.path.join(d, "spec.json"), "w") as fh:
            json.dump({"complement": bool(complement), "semiring": sr, "reps": int(reps), "threads": threads,
                       "one_thread_rows": True, "sample": bool(sample)}, fh)
        env = dict(os.environ, OMP_PROC_BIND="close")
        res = subprocess.run([sys.executable, "-m", "oracle.bench_leg", d], env=env, cwd=ROOT, capture_output=True,
                             text=True, timeout=900)
        if res.returncode != 0:
            raise RuntimeError(f"oracle CPU leg failed: {res.stderr[-2000:]}")
        rep = json.loads(res.stdout.strip().splitlines()[-1])
        rep["affinity_cores"], rep["cgroup_cpu_quota"] = aff, quota
        if sample:
            rep["C"] = tuple(np.load(os.path.join(d, f"C_{x}.npy")) for x in ("rowptr", "colidx", "values"))
        return rep
    finally:
        shutil.rmtree(d, ignore_errors=True)


def baseline_record(rep, sample_desc):
    """cpu_baseline entry from a CPU-leg report: useful GFLOP/s of the sample
    at the best thread count (median of the runs), and on one thread."""
    med = {int(nt): float(np.median(ts)) for nt, ts in rep["runs"].items()}
    nt = min(med, key=med.get)
    t = med[nt]
    one = rep.get("one_thread")
    reps = len(next(iter(rep["runs"].values())))
    return {"value": sig(2 * rep["useful"] / t / 1e9), "unit": "GFLOP/s", "cores": nt, "kind": "oracle",
            "sample": f"{sample_desc}; median of {reps} runs of {t:.3f} s on {nt} threads (OMP_PROC_BIND=close)",
            "one_thread_value": sig(2 * one["useful"] / one["seconds"] / 1e9) if one else None,
            "one_thread_sample_rows": one["rows"] if one else None,
            "seconds_by_threads": {str(k): round(v, 4) for k, v in med.items()},
            "affinity_cores": rep["affinity_cores"], "cgroup_cpu_quota": rep["cgroup_cpu_quota"],
            "cpu_model": cpu_model()}


def gather_rows(rp, ci, v, rows):
    """Rows `rows` of a host CSR as (rowptr, colidx, values)."""
    rows = np.asarray(rows, np.int64)
    lens = rp[rows + 1] - rp[rows]
    out_rp = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(lens, out=out_rp[1:])
    idx = np.repeat(rp[rows] - out_rp[:-1], lens) + np.arange(int(out_rp[-1]), dtype=np.int64)
    return out_rp, ci[idx], v[idx]


def same_rows(got, exp, fp64):
    """Patterns exactly; values exactly, or within 1e-12 relative for FP64."""
    if not (np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1])):
        return False
    if fp64:
        return bool(np.all(np.abs(got[2] - exp[2]) <= 1e-12 * np.abs(exp[2])))
    return np.array_equal(got[2], exp[2])


def row_flops(A, Bdeg):
    """flops_i = sum over k in A(i,:) of nnz(B(k,:)) for every row i."""
    rows = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
    return np.bincount(rows, weights=Bdeg[A.colidx], minlength=A.nrows).astype(np.int64)


def time_steps(dA, dB, dM, comp, sr, steps, warmup, kw, post=None):
    """Times `steps` whole steps (plan creation, execution, and `post`) after
    `warmup` untimed ones. The warm-up steps time every kernel bin to find
    the dominant one; the timed steps record HIP events on the dominant
    bin's launches only (an event pair costs the step several microseconds)
    into a timing session read after them. The other stages come from
    untimed profiled executions. Returns a dict with the step time, stage
    times per step, plan-creation and cold-step times and the last step's
    output (device tensors)."""
    import torch

    import paper_2111_09947_amd as msp
    dev = dA.rowptr.device
    odt = msp.out_dtype(sr)
    stage_ms = np.zeros(len(msp.STAGE_NAMES), dtype=np.float64)
    timing = msp.Timing(max(warmup, 1), stages=msp.BIN_NAMES)

    def step(timed=True):
        with msp.Plan(dA, dB, dM, complement=comp, semiring=sr, **kw) as p:  # the plan's one synchronization
            cap = max(p.upper_bound, 1)
            rp = torch.empty(dA.nrows + 1, dtype=torch.int64, device=dev)
            ci = torch.empty(cap, dtype=torch.int32, device=dev)
            v = torch.empty(cap, dtype=odt, device=dev)
            if timed:
                p.execute_timed(rp, ci, v, cap, timing)
            else:
                p.execute_into(rp, ci, v, cap)
            if post is not None:
                post(rp, v)
            return rp, ci, v

    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    warm_ms = timing.collect(np.zeros_like(stage_ms))
    timing.close()
    dom = int(np.argmax(warm_ms[:len(msp.BIN_NAMES)]))
    timing = msp.Timing(steps, stages=[msp.BIN_NAMES[dom]])
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    timing.collect(stage_ms)
    timing.close()
    other_stages(lambda: msp.Plan(dA, dB, dM, complement=comp, semiring=sr, **kw), dA.nrows, odt, stage_ms, steps,
                 dev, keep=dom)
    plan_ms = []
    for _ in range(3):  # plan creation alone (in a step it also waits for the previous step)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        msp.Plan(dA, dB, dM, complement=comp, semiring=sr, **kw).close()
        plan_ms.append((time.perf_counter() - c0) * 1e3)
    # cold steps: L2 and the last-level cache flushed by writing 512 MiB before each one
    flush = torch.empty(1 << 26, dtype=torch.int64, device=dev)
    cold_ms = []
    for r in range(5):
        flush.fill_(r)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        step(False)
        torch.cuda.synchronize()
        cold_ms.append((time.perf_counter() - c0) * 1e3)
    del flush
    with msp.Plan(dA, dB, dM, complement=comp, semiring=sr, **kw) as p:
        bins, bin_units, products = p.row_bins(), p.bin_units, p.products
    return {"ms": ms, "stage_ms": stage_ms / steps, "dom": dom, "plan_ms": float(np.median(plan_ms)),
            "cold_ms": float(np.median(cold_ms)), "out": out, "bins": bins, "bin_units": bin_units,
            "products": int(products)}


def useful_rows(dA, dB, dM, comp):
    """Admitted products per row: the plus-pair product's row sums."""
    import paper_2111_09947_amd as msp
    with msp.Plan(dA, dB, dM, complement=comp, semiring="plus_pair_i64") as p:
        C = p.execute()
    rp = C.rowptr.cpu().numpy()
    owner = np.repeat(np.arange(dA.nrows), np.diff(rp))
    return np.bincount(owner, weights=C.values.cpu().numpy(), minlength=dA.nrows).astype(np.int64)


def roofline_record(t, per_row, traffic_key):
    """The dominant kernel bin (largest time per step, timed live in the
    timed steps): its rows' algorithmic bytes per launch over its HIP-event
    time, against the HBM peak; the counter-measured HBM bytes per launch
    (calibrated, same kernel source) when a traffic summary exists for it."""
    import paper_2111_09947_amd as msp
    bin_ms = t["stage_ms"][:len(msp.BIN_NAMES)]
    dom = t["dom"]
    name = msp.BIN_NAMES[dom]
    dom_bytes = int(per_row[t["bins"] == dom].sum())
    dom_ms = float(bin_ms[dom])
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    traffic = load_traffic(os.path.join(ROOT, "profiles", f"traffic_{traffic_key}.json"), kernel_source_hash(), name)
    rec = {"bound": "hbm", "achieved": sig(achieved), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": sig(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": f"numeric bin {name}",
           "kernel_ms": round(dom_ms, 5), "alg_bytes": dom_bytes}
    if traffic:
        # the rate the HBM counters saw (the kernel is limited by issue and cache, not by HBM, when it is low)
        rec["traffic_gbs"] = round(traffic / (dom_ms * 1e-3) / 1e9, 1)
        rec["traffic_frac"] = round(traffic / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return rec


def product_record(t, per_row, useful, traffic_key, bytes_min):
    import paper_2111_09947_amd as msp
    ms = t["ms"]
    total = int(per_row.sum())
    return {
        "ms_per_step": round(ms, 4),
        "value": sig(2 * useful / (ms * 1e-3) / 1e9), "unit": "GFLOP/s",
        "products": t["products"], "useful_products": int(useful),
        "bin_units": t["bin_units"],
        "roofline": roofline_record(t, per_row, traffic_key),
        "path": {
            "alg_bytes_total": total,
            "hbm_frac_whole_step": sig(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "stage_ms": {n: round(float(x), 5) for n, x in zip(msp.STAGE_NAMES, t["stage_ms"]) if x > 0},
            "plan_create_ms": round(t["plan_ms"], 4),
            "cold_ms_per_step": round(t["cold_ms"], 4),
            "bytes_min": int(bytes_min),
        },
    }


def measure_er(args):
    """Erdos-Renyi A, B, M, n = 4096, average degree 8, uniform columns, FP64
    U(0,1) values, plus-times, normal mask (seeds 101, 102, 103). Whole output
    checked against the oracle."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp
    dev = torch.device("cuda:0")
    n, d = 4096, 8.0
    A = mspgen.er(n, n, d, 101, "f64")
    B = mspgen.er(n, n, d, 102, "f64")
    M = mspgen.er(n, n, d, 103, None)
    sr = "plus_times_f64"
    dA = msp.DeviceCSR.from_host(A, dev, torch.float64)
    dB = msp.DeviceCSR.from_host(B, dev, torch.float64)
    dM = msp.DeviceCSR.from_host(M, dev)
    t = time_steps(dA, dB, dM, False, sr, args.steps, args.warmup, tuning_kw(args))
    rp, ci, v = t["out"]
    nnz = int(rp[-1].item())
    got = (rp.cpu().numpy(), ci[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
    useful_row = useful_rows(dA, dB, dM, False)
    per_row = alg_bytes(np.diff(A.rowptr), row_flops(A, np.diff(B.rowptr)), np.diff(M.rowptr), useful_row,
                        np.diff(got[0]), wA=8, wB=8, wC=8)
    rec = {"workload": "Erdos-Renyi A, B, M: n = 4096, average degree 8 (uniform columns), FP64 U(0,1), "
                       "plus-times, normal mask; seeds 101, 102, 103",
           "dtype": "f64", "n": n, "nnz_A": A.nnz, "nnz_B": B.nnz, "nnz_M": M.nnz, "nnz_C": nnz,
           **product_record(t, per_row, int(useful_row.sum()), "er4096",
                            3 * (8 * (n + 1)) + 12 * (A.nnz + B.nnz) + 4 * M.nnz + 12 * nnz)}
    if not args.no_cpu_baseline:
        rep = cpu_leg(A, B, M, False, sr, reps=5, sample=True)
        ok = same_rows(got, rep["C"], True)
        rec["parity"] = {"checked": "every row against the oracle", "identical_within_tolerance": ok}
        if not ok:
            print("[bench] MISMATCH: Erdos-Renyi n=4096 differs from the oracle", file=sys.stderr)
            sys.exit(1)
        rec["cpu_baseline"] = baseline_record(rep, "the whole product")
    return rec


def measure_complement(args):
    """Erdos-Renyi A (2^16 x 2^20) and B (2^20 x 2^20) of average degree 16,
    FP64 U(0,1) values, plus-times, under a complemented Erdos-Renyi mask of
    degree 8 (seeds 41, 42, 43): the regime of complemented masks wider than
    one dense tile, where rows of more than heap_flops products are sorted.
    Every 4th row checked against the oracle."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp
    dev = torch.device("cuda:0")
    m, n, d, dm = 1 << 16, 1 << 20, 16.0, 8.0
    A = mspgen.er(m, n, d, 41, "f64")
    B = mspgen.er(n, n, d, 42, "f64")
    M = mspgen.er(m, n, dm, 43, None)
    sr = "plus_times_f64"
    dA = msp.DeviceCSR.from_host(A, dev, torch.float64)
    dB = msp.DeviceCSR.from_host(B, dev, torch.float64)
    dM = msp.DeviceCSR.from_host(M, dev)
    t = time_steps(dA, dB, dM, True, sr, args.steps, args.warmup, tuning_kw(args))
    rp, ci, v = t["out"]
    nnz = int(rp[-1].item())
    got = (rp.cpu().numpy(), ci[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
    del t["out"], rp, ci, v
    useful_row = useful_rows(dA, dB, dM, True)
    per_row = alg_bytes(np.diff(A.rowptr), row_flops(A, np.diff(B.rowptr)), np.diff(M.rowptr), useful_row,
                        np.diff(got[0]), wA=8, wB=8, wC=8)
    rec = {"workload": "Erdos-Renyi A 2^16 x 2^20 and B 2^20 x 2^20, average degree 16, FP64 U(0,1), plus-times, "
                       "complemented Erdos-Renyi mask of degree 8; seeds 41, 42, 43",
           "dtype": "f64", "m": m, "n": n, "nnz_A": A.nnz, "nnz_B": B.nnz, "nnz_M": M.nnz, "nnz_C": nnz,
           **product_record(t, per_row, int(useful_row.sum()), "complement_er2p20",
                            8 * (m + 1) * 3 + 8 * (n + 1) + 12 * (A.nnz + B.nnz) + 4 * M.nnz + 12 * nnz)}
    if not args.no_cpu_baseline:
        rep = cpu_leg(A, B, M, True, sr, reps=3, sample=True)
        ok = same_rows(got, rep["C"], True)
        rec["parity"] = {"checked": "every row against the oracle", "identical_within_tolerance": ok}
        if not ok:
            print("[bench] MISMATCH: the complemented product differs from the oracle", file=sys.stderr)
            sys.exit(1)
        rec["cpu_baseline"] = baseline_record(rep, "the whole product")
    return rec


def measure_er_batched(args, count=256):
    """`count` independent Erdos-Renyi products of the n = 4096 shape (product
    p: seeds 101 + 10p, 102 + 10p, 103 + 10p; product 0 is the single
    product above) as one batch: the single product is bound by launch and
    synchronization latency (its 2.2 MB of algorithmic bytes take 0.28 us
    at the HBM peak), so its throughput shape is many of them per launch.
    Times one whole step (batch plan creation with its synchronization,
    binding, execution) and, separately, replays of the captured graph.
    Products 0, 1 and the last are checked against the oracle in full."""
    import torch

    import mspgen
    import oracle
    import paper_2111_09947_amd as msp
    dev = torch.device("cuda:0")
    n, d, sr = 4096, 8.0, "plus_times_f64"
    host, probs = [], []
    for p in range(count):
        A = mspgen.er(n, n, d, 101 + 10 * p, "f64")
        B = mspgen.er(n, n, d, 102 + 10 * p, "f64")
        M = mspgen.er(n, n, d, 103 + 10 * p, None)
        host.append((A, B, M))
        probs.append((msp.DeviceCSR.from_host(A, dev, torch.float64), msp.DeviceCSR.from_host(B, dev, torch.float64),
                      msp.DeviceCSR.from_host(M, dev), False))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        def step():
            with msp.Batch(probs, semiring=sr) as b:
                b.bind_new_outputs()
                b.execute()
                return b.results(), b.bin_units, int(sum(b.products))
        ms_step = _timed(step, args.steps, args.warmup)
        res, bin_units, products = step()
        b = msp.Batch(probs, semiring=sr)
        b.bind_new_outputs()
        ms_graph = _timed(b.graph_launch, args.steps, args.warmup)
        stage_ms = np.zeros(len(msp.STAGE_NAMES))
        timing = msp.Timing(args.steps, stages=msp.BIN_NAMES)
        for _ in range(args.steps):
            b.execute_timed(timing)
        timing.collect(stage_ms)
        timing.close()
        stage_ms /= args.steps
        bins = b.row_bins()
        b.close()
        with msp.Batch(probs, semiring="plus_pair_i64") as bp:
            bp.bind_new_outputs()
            bp.execute()
            pair = bp.results()
    per_row, useful = [], 0
    for (A, B, M), Cp, C in zip(host, pair, res):
        prp = Cp.rowptr.cpu().numpy()
        owner = np.repeat(np.arange(n), np.diff(prp))
        u_row = np.bincount(owner, weights=Cp.values.cpu().numpy(), minlength=n).astype(np.int64)
        useful += int(u_row.sum())
        per_row.append(alg_bytes(np.diff(A.rowptr), row_flops(A, np.diff(B.rowptr)), np.diff(M.rowptr), u_row,
                                 np.diff(C.rowptr.cpu().numpy()), wA=8, wB=8, wC=8))
    per_row = np.concatenate(per_row)
    ok = True
    for p in (0, 1, count - 1):
        A, B, M = host[p]
        R = oracle.masked_spgemm(A, B, M, False, sr)
        ok = ok and same_rows(tuple(x.cpu().numpy() for x in (res[p].rowptr, res[p].colidx, res[p].values)),
                              (R.rowptr, R.colidx, R.values), True)
    if not ok:
        print("[bench] MISMATCH: batched Erdos-Renyi products differ from the oracle", file=sys.stderr)
        sys.exit(1)
    bin_ms = stage_ms[:len(msp.BIN_NAMES)]
    dom = int(np.argmax(bin_ms))
    dom_bytes = int(per_row[bins == dom].sum())
    achieved = dom_bytes / (bin_ms[dom] * 1e-3) / 1e9 if bin_ms[dom] > 0 else 0.0
    total = int(per_row.sum())
    roof = {"bound": "hbm", "achieved": sig(achieved), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": sig(achieved / HBM_PEAK_GBS, 4),
            "traffic": load_traffic(os.path.join(ROOT, "profiles", "traffic_er4096_x256.json"), kernel_source_hash(),
                                    msp.BIN_NAMES[dom]),
            "kernel": f"numeric bin {msp.BIN_NAMES[dom]}", "kernel_ms": round(float(bin_ms[dom]), 5),
            "alg_bytes": dom_bytes}
    if roof["traffic"] and bin_ms[dom] > 0:
        roof["traffic_gbs"] = round(roof["traffic"] / (bin_ms[dom] * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_gbs"] / HBM_PEAK_GBS, 4)
    return {"workload": f"{count} independent Erdos-Renyi products of the n = 4096, average degree 8, FP64 "
                        "plus-times shape (product p: seeds 101+10p, 102+10p, 103+10p) as one batch",
            "dtype": "f64", "products": products, "useful_products": useful, "bin_units": bin_units,
            "ms_per_step": round(ms_step, 4), "value": sig(2 * useful / (ms_step * 1e-3) / 1e9), "unit": "GFLOP/s",
            "graph_replay_ms": round(ms_graph, 4),
            "roofline": roof,
            "path": {"alg_bytes_total": total,
                     "hbm_frac_whole_step": sig(total / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "hbm_frac_graph_replay": sig(total / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "stage_ms": {nm: round(float(x), 5) for nm, x in zip(msp.STAGE_NAMES, stage_ms) if x > 0}},
            "parity": {"checked": f"products 0, 1 and {count - 1} in full against the oracle",
                       "identical_within_tolerance": ok}}


def measure_tc(args):
    """Triangle counting: R-MAT scale 18, edge factor 16, symmetrized,
    degree-relabelled, L = strict lower triangle; C = L .* (L L) under
    plus-pair (int64), then the sum of C."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp

    dev = torch.device("cuda:0")
    t0 = time.time()
    L = mspgen.triangle_input(args.scale, args.edge_factor, args.seed)
    print(f"[bench] tc input: R-MAT scale {args.scale} ef {args.edge_factor}: n={L.nrows} nnz(L)={L.nnz} "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    dL = msp.DeviceCSR.from_host(L, dev)
    sr = "plus_pair_i64"
    total_dev = torch.empty(1, dtype=torch.int64, device=dev)
    kw = dict(phase=args.phase, force_kind=args.force_kind, inner_ratio=args.inner_ratio, **tuning_kw(args))
    t = time_steps(dL, dL, dL, False, sr, args.steps, args.warmup, kw,
                   post=lambda rp, v: msp.reduce_csr(rp, L.nrows, v, sr, out=total_dev))
    rp, ci, v = t["out"]
    nnz = int(rp[-1].item())
    triangles = int(total_dev.item())
    got = (rp.cpu().numpy(), ci[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
    owner = np.repeat(np.arange(L.nrows), np.diff(got[0]))
    useful_row = np.bincount(owner, weights=got[2], minlength=L.nrows).astype(np.int64)
    assert int(useful_row.sum()) == triangles
    deg = np.diff(L.rowptr)
    per_row = alg_bytes(deg, row_flops(L, deg), deg, useful_row, np.diff(got[0]))
    rec = {"workload": f"triangle counting C = L .* (L L), plus-pair int64, then sum; R-MAT scale {args.scale} "
                       f"edge factor {args.edge_factor} (a,b,c = .57,.19,.19), symmetrized, degree-relabelled, "
                       "L = strict lower triangle",
           "dtype": "int64", "n": L.nrows, "nnz_L": L.nnz, "nnz_C": nnz, "triangles": triangles,
           "phase": args.phase, "kind": args.force_kind or "auto",
           **product_record(t, per_row, triangles, "tc_rmat18",
                            3 * (8 * (L.nrows + 1) + 4 * L.nnz) + 8 * (L.nrows + 1) + 12 * nnz)}
    if not args.no_cpu_baseline:
        rep = cpu_leg(L, L, L, False, sr, reps=5, sample=True)
        ok = rep["sum"] == triangles and same_rows(got, rep["C"], False)
        rec["parity"] = {"checked": "every row and the triangle count against the oracle", "identical": ok}
        if not ok:
            print(f"[bench] MISMATCH: oracle {rep['sum']} triangles, GPU {triangles}", file=sys.stderr)
            sys.exit(1)
        rec["cpu_baseline"] = baseline_record(rep, "the whole workload (masked product + sum)")
    return rec


def measure_bfs(args):
    """One multi-source BFS step: R-MAT scale 20, edge factor 16, 512 sources
    at depths 1..3; C = !V .* (A F) with A the symmetric graph, F the frontiers
    (n x 512) and V the visited sets, under the int32 path-count semiring
    (plus-times, wrapping) and the boolean semiring. Returns one record per
    semiring."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp

    dev = torch.device("cuda:0")
    t0 = time.time()
    G = mspgen.rmat_graph(20, 16, 20)
    print(f"[bench] bfs graph: R-MAT scale 20 ef 16: n={G.nrows} nnz={G.nnz} ({time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)
    F64, V, srcs, lv = mspgen.bfs_step_input(G, 512, 21, "i64")
    print(f"[bench] bfs frontiers ({time.time() - t0:.1f}s): nnz(F)={F64.nnz} nnz(V)={V.nnz}", file=sys.stderr,
          flush=True)
    n = G.nrows
    dA = msp.DeviceCSR.from_host(G, dev)
    dV = msp.DeviceCSR.from_host(V, dev)
    nnzA = np.diff(G.rowptr)
    flops = row_flops(G, np.diff(F64.rowptr))
    mnnz = np.diff(V.rowptr)
    out = {}
    useful_row = None
    for sr, F, w in (("plus_times_i32", F64.with_values(F64.values.astype(np.int32)), 4),
                     ("lor_land_bool", F64.with_values(np.ones(F64.nnz, np.uint8)), 1)):
        dF = msp.DeviceCSR.from_host(F, dev, msp.in_dtype(sr))
        t = time_steps(dA, dF, dV, True, sr, args.steps, args.warmup, tuning_kw(args))
        rp, ci, v = t["out"]
        nnz = int(rp[-1].item())
        got = (rp.cpu().numpy(), ci[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())
        del t["out"], rp, ci, v
        if useful_row is None:
            useful_row = useful_rows(dA, dF, dV, True)
        per_row = alg_bytes(nnzA, flops, mnnz, useful_row, np.diff(got[0]), wA=0, wB=w, wC=w)
        rec = {"workload": "multi-source BFS step C = !V .* (A F): R-MAT scale 20 edge factor 16 "
                           "(a,b,c = .57,.19,.19, symmetrized), 512 sources at depth 1..3, complemented visited "
                           f"mask; {'int32 path counts' if w == 4 else 'boolean'}",
               "dtype": "int32" if w == 4 else "u8", "n": n, "nnz_A": G.nnz, "nnz_F": F.nnz, "nnz_V": V.nnz,
               "nnz_C": nnz,
               **product_record(t, per_row, int(useful_row.sum()), f"bfs_rmat20_{'i32' if w == 4 else 'bool'}",
                                8 * (n + 1) * 4 + 4 * G.nnz + (4 + w) * F.nnz + 4 * V.nnz + (4 + w) * nnz)}
        if not args.no_cpu_baseline:
            stride = 4 if w == 4 else 16
            rows = np.arange(0, n, stride, dtype=np.int64)
            rep = cpu_leg(G, F, V, True, sr, rows=rows, rows_one=np.arange(0, n, 64, dtype=np.int64),
                          reps=3 if w == 4 else 1, sample=True)
            ok = same_rows(gather_rows(*got, rows), rep["C"], False)
            rec["parity"] = {"checked": f"every {stride}th row ({len(rows)} rows) against the oracle",
                             "identical": ok}
            if not ok:
                print(f"[bench] MISMATCH: BFS step ({sr}) differs from the oracle", file=sys.stderr)
                sys.exit(1)
            rec["cpu_baseline"] = baseline_record(rep, f"every {stride}th row of the step ({len(rows)} rows)")
        out[sr] = rec
        del dF
        torch.cuda.empty_cache()
    return out


def headline(rec, args, extra=None):
    """The JSON line around one workload record."""
    line = {"metric": "useful_masked_gflops", "value": rec["value"], "unit": "GFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": rec["dtype"],
            "data": "synthetic",
            "config": {k: v for k, v in rec.items() if k not in ("value", "unit", "ms_per_step", "roofline",
                                                                 "path", "cpu_baseline", "dtype")},
            "roofline": rec["roofline"], "path": rec["path"], "cpu_baseline": rec.get("cpu_baseline")}
    if extra:
        line.update(extra)
    return line


def run_tc(args):
    print(json.dumps(headline(measure_tc(args), args)), flush=True)


def run_er(args):
    print(json.dumps(headline(measure_er(args), args)), flush=True)


def run_bfs(args):
    recs = measure_bfs(args)
    print(json.dumps(headline(recs["plus_times_i32"], args, {"semirings": recs})), flush=True)


def run_all(args):
    """The default run: the multi-source BFS step (the largest single-GPU
    workload, int32 path counts: the headline value), with the triangle
    count and the Erdos-Renyi n = 4096 product as further records, each with
    its own roofline, whole-step fraction, oracle check and CPU baseline."""
    import torch
    dev = torch.device("cuda:0")
    bfs = measure_bfs(args)
    torch.cuda.empty_cache()
    tc = measure_tc(args)
    torch.cuda.empty_cache()
    er = measure_er(args)
    torch.cuda.empty_cache()
    er_batched = measure_er_batched(args)
    line = headline(bfs["plus_times_i32"], args, {
        "device": device_info(dev),
        "workloads": {"bfs_rmat20_i32": bfs["plus_times_i32"], "bfs_rmat20_bool": bfs["lor_land_bool"],
                      "tc_rmat18": tc, "er4096_f64": er, "er4096_f64_x256_batched": er_batched}})
    print(json.dumps(line), flush=True)


def run_bc(args):
    """Batched betweenness-centrality dependencies: 512 random non-isolated
    sources on the symmetric R-MAT graph (scale --scale, edge factor
    --edge-factor), the whole two-stage computation (forward multi-source BFS
    with complemented masks, backward sweep with normal masks) per step.
    Metric: TEPS = batch x undirected edges / time (Section "Betweenness
    Centrality")."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp

    dev = torch.device("cuda:0")
    t0 = time.time()
    G = mspgen.rmat_graph(args.scale, args.edge_factor, 20)
    deg = np.diff(G.rowptr)
    rng = np.random.default_rng(21)
    srcs = rng.choice(np.nonzero(deg > 0)[0], size=512, replace=False).astype(np.int32)
    dG = msp.DeviceCSR.from_host(G.with_values(None), dev)
    edges = G.nnz // 2
    print(f"[bench] bc input: R-MAT scale {args.scale} ef {args.edge_factor}: n={G.nrows} undirected edges={edges} "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    bc = torch.zeros(G.nrows, dtype=torch.float64, device=dev)
    info = None
    for _ in range(args.warmup):
        bc.zero_()
        _, info = msp.bc_batch(dG, srcs, bc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwd = bwd = 0.0
    for _ in range(args.steps):
        bc.zero_()
        _, info = msp.bc_batch(dG, srcs, bc)
        fwd += info["forward_ms"]
        bwd += info["backward_ms"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) / args.steps * 1e3
    teps = 512 * edges / (ms * 1e-3)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = min(16, len(os.sched_getaffinity(0)))
        k = 64
        c0 = time.perf_counter()
        ref = oracle.bc(G, srcs[:k], nthreads=nthreads)
        t_cpu = time.perf_counter() - c0
        bc.zero_()
        got, _ = msp.bc_batch(dG, srcs[:k], bc)
        err = float(np.max(np.abs(got.cpu().numpy() - ref) / np.maximum(np.abs(ref), 1.0)))
        if err > 1e-9:
            print(f"[bench] MISMATCH against the oracle: max relative error {err:.3g}", file=sys.stderr)
            sys.exit(1)
        cpu = {"value": round(k * edges / t_cpu / 1e6, 2), "unit": "MTEPS", "cores": nthreads, "kind": "oracle",
               "sample": f"{k} of the 512 sources (Brandes per source), {t_cpu:.2f} s; checked against the GPU "
                         f"result for the same {k} sources (max relative error {err:.2g})"}
    out = {
        "metric": "bc_mteps", "value": round(teps / 1e6, 1), "unit": "MTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"betweenness-centrality dependencies, 512 sources, R-MAT scale {args.scale} edge "
                               f"factor {args.edge_factor} (symmetrized)", "n": G.nrows, "undirected_edges": edges,
                   **info},
        "stages_ms": {"forward": round(fwd / args.steps, 3), "backward": round(bwd / args.steps, 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_ktruss(args):
    """5-truss of the symmetric R-MAT graph (scale --scale, edge factor
    --edge-factor) by repeated masked products with pruning. Metric as in
    Section "k-truss": the flops of all masked products (2 per product)
    divided by the total time of the whole computation."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp

    dev = torch.device("cuda:0")
    k = 5
    G = mspgen.rmat_graph(args.scale, args.edge_factor, 18)
    dG = msp.DeviceCSR.from_host(G.with_values(None), dev)
    info = None
    for _ in range(args.warmup):
        C, info = msp.ktruss(dG, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        C, info = msp.ktruss(dG, k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) / args.steps * 1e3
    value = 2 * info["products"] / (ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = time.perf_counter()
        erp, eci, esup = oracle.ktruss(G, k)
        t_cpu = time.perf_counter() - c0
        rp, ci, sup = C.to_host()
        if not (np.array_equal(rp, erp) and np.array_equal(ci, eci) and np.array_equal(sup, esup)):
            print("[bench] MISMATCH: the GPU truss differs from the oracle's", file=sys.stderr)
            sys.exit(1)
        cpu = {"value": round(2 * info["products"] / t_cpu / 1e9, 3), "unit": "GFLOP/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"the whole {k}-truss ({t_cpu:.2f} s), result identical to the GPU's"}
    out = {
        "metric": "ktruss_gflops", "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"{k}-truss, R-MAT scale {args.scale} edge factor {args.edge_factor} (symmetrized)",
                   "n": G.nrows, "nnz": G.nnz, "truss_nnz": int(C.colidx.numel()), **info},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_heatmap(args):
    """Best accumulator kind against input and mask density (the GPU analogue
    of Section "Effect of Input Matrix and Mask Density"): Erdos-Renyi A, B
    (degree d) and M (degree dm), n = 2^12 .. 2^22, FP64 plus-times, normal
    mask. Every kind (and the automatic binner) runs the whole product (plan
    creation included; the inner kind builds B^T inside it), best of 3; all
    kinds must give the same result (pattern exact, values within 1e-12),
    and 64 sampled rows of every cell are checked against the oracle. Cells
    with more than 2^31 products or mask entries are skipped, the dense kind
    is run only up to n = 2^14 (its 4096-column tiles restream a row once per
    tile), the heap kind only for d <= 4 (rows of A with more than 8 entries
    leave it), and mask degree 1024 only up to n = 2^18.

    Then the binner thresholds are tuned on the heatmap: every cell runs the
    automatic binner under each setting of a grid of maskidx_max (the
    search/hash split for mask rows), heap_flops and block_flops, and the
    setting with the smallest geometric mean of (automatic time / best forced
    time) over the cells is reported beside the library's defaults."""
    import itertools

    import torch

    import mspgen
    import oracle
    import paper_2111_09947_amd as msp

    dev = torch.device("cuda:0")
    kinds = [None, "dense", "hash", "maskidx", "inner", "heap"]
    space = {"maskidx_max": [0, 8, 64], "heap_flops": [0, 32, 128], "block_flops": [2048, 8192, 32768]}
    settings = [dict(zip(space, v)) for v in itertools.product(*space.values())]
    grid = []
    rng = np.random.default_rng(12)

    def best_of(fn, reps):
        best = float("inf")
        out = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t) * 1e3)
        return best, out

    for lg in (12, 14, 16, 18, 20, 22):
        n = 1 << lg
        for d in (1, 4, 16, 64):
            if n * d * d > (1 << 31):
                continue
            hA = mspgen.er(n, n, d, 1000 + lg, "f64")
            hB = mspgen.er(n, n, d, 2000 + lg, "f64")
            A = msp.DeviceCSR.from_host(hA, dev, torch.float64)
            B = msp.DeviceCSR.from_host(hB, dev, torch.float64)
            for dm in (1, 4, 16, 64, 256, 1024):
                if (dm == 1024 and lg > 18) or n * dm > (1 << 31):
                    continue
                hM = mspgen.er(n, n, dm, 3000 + lg, None)
                M = msp.DeviceCSR.from_host(hM, dev)
                cell = {"n": n, "d": d, "dm": dm, "ms": {}}
                ref = None
                for kind in kinds:
                    if (kind == "dense" and lg > 14) or (kind == "heap" and d > 4):
                        continue
                    t, C = best_of(lambda: msp.masked_spgemm(A, B, M, semiring="plus_times_f64", force_kind=kind), 3)
                    h = C.to_host()
                    if ref is None:
                        ref = h
                        rows = np.unique(rng.integers(0, n, 64))
                        R = oracle.masked_spgemm(hA, hB, hM, False, "plus_times_f64", rows=rows)
                        if not same_rows(gather_rows(*h, rows), (R.rowptr, R.colidx, R.values), True):
                            print(f"[bench] MISMATCH against the oracle n={n} d={d} dm={dm}", file=sys.stderr)
                            sys.exit(1)
                    elif not same_rows(h, ref, True):
                        print(f"[bench] MISMATCH kind={kind} n={n} d={d} dm={dm}", file=sys.stderr)
                        sys.exit(1)
                    cell["ms"][kind or "auto"] = round(t, 4)
                forced = {k: v for k, v in cell["ms"].items() if k != "auto"}
                cell["best"] = min(forced, key=forced.get)
                cell["auto_over_best"] = round(cell["ms"]["auto"] / forced[cell["best"]], 3)
                # the automatic binner under every threshold setting of the grid
                cell["tuning_ms"] = [round(best_of(lambda: msp.masked_spgemm(A, B, M, semiring="plus_times_f64",
                                                                             **st), 2)[0], 4) for st in settings]
                grid.append(cell)
                print(f"[bench] n=2^{lg} d={d} dm={dm}: best {cell['best']} {cell['ms']}", file=sys.stderr,
                      flush=True)
                del M, hM
            del A, B, hA, hB
            torch.cuda.empty_cache()
    best_forced = np.array([min(v for k, v in c["ms"].items() if k != "auto") for c in grid])
    tun = np.array([c["tuning_ms"] for c in grid])  # cells x settings
    geo = np.exp(np.mean(np.log(tun / best_forced[:, None]), axis=0))
    k_best = int(np.argmin(geo))
    defaults = {"maskidx_max": 8, "heap_flops": 32, "block_flops": 8192}
    k_def = settings.index(defaults)
    ratios = [c["auto_over_best"] for c in grid]
    out = {"metric": "heatmap_auto_over_best_median", "value": round(float(np.median(ratios)), 3),
           "unit": "ratio", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "ER n=2^12..2^22, input degree 1..64, mask degree 1..1024, FP64 plus-times"},
           "worst_auto_over_best": round(float(np.max(ratios)), 3),
           "thresholds": {"space": space, "settings": settings,
                          "geomean_auto_over_best": [round(float(g), 4) for g in geo],
                          "best": settings[k_best], "best_geomean": round(float(geo[k_best]), 4),
                          "defaults": defaults, "defaults_geomean": round(float(geo[k_def]), 4)},
           "cells": [{k: v for k, v in c.items() if k != "tuning_ms"} for c in grid]}
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Poisson stream of masked products drawn uniformly from a pool of the
    benchmark shapes (Erdos-Renyi n = 4096 with fresh seeds, triangle counting
    on R-MAT scale 18, the 512-source BFS step on R-MAT scale 20, and the 64
    mixed products at full size), plus-pair int64 for
    triangle counting and 50/50 plus-pair int64 or FP64 plus-times otherwise;
    operands resident on the GPU. Arrival rate = 0.8 x the capacity measured
    in a closed loop. Continuous batching (slots on their own streams, same-
    semiring mini-batches, memory admission) against a FIFO server that runs
    one product at a time."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp
    from paper_2111_09947_amd import serve
    from paper_2111_09947_amd.autotune import same_output

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    t0 = time.time()

    def up(X, f64):
        return msp.DeviceCSR.from_host(X, dev, torch.float64 if f64 else None)

    pool = []
    for s in range(4):
        A = mspgen.er(4096, 4096, 8.0, 101 + 10 * s, "f64")
        B = mspgen.er(4096, 4096, 8.0, 102 + 10 * s, "f64")
        M = mspgen.er(4096, 4096, 8.0, 103 + 10 * s, None)
        pool.append(dict(name="er4096", ops=(up(A, True), up(B, True), up(M, False), False), f64=True))
    L = mspgen.triangle_input(18, 16, 18)
    dL = up(L, False)
    pool.append(dict(name="tc_rmat18", ops=(dL, dL, dL, False), f64=False))
    G = mspgen.rmat_graph(20, 16, 20)
    F, V, _, _ = mspgen.bfs_step_input(G, 512, 21, "i64")
    F = F.with_values(F.values.astype(np.float64))
    G = G.with_values(np.ones(G.nnz))
    pool.append(dict(name="bfs_rmat20", ops=(up(G, True), up(F, True), up(V, False), True), f64=True))
    del G, F, V
    for prm in mspgen.batch_params(64, seed=4):  # full-size masks, uploaded product by product
        A, B = mspgen.batch_operands(prm)
        M = mspgen.batch_mask(prm)
        pool.append(dict(name=f"mix{prm['t']}", ops=(up(A, True), up(B, True), up(M, False), False), f64=True))
        del A, B, M
    print(f"[bench] serving pool of {len(pool)} items ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    for it in pool:  # admitted-product count per item (semiring independent)
        A, B, M, c = it["ops"]
        with msp.Plan(A, B, M, complement=c, semiring="plus_pair_i64") as p:
            C = p.execute()
            it["useful"] = int(C.values.sum().item())
        it["bytes"] = {sr: serve.product_bytes(A, B, M, c, sr) for sr in ("plus_pair_i64", "plus_times_f64")}
        it["work"] = serve.product_info(A, B, M, c, "plus_pair_i64")[1]

    def draw(n, seed):
        r = np.random.default_rng(seed)
        items = r.integers(0, len(pool), size=n)
        coin = r.random(n) < 0.5
        return [(int(k), "plus_pair_i64" if (not pool[k]["f64"] or coin[x]) else "plus_times_f64")
                for x, k in enumerate(items)]

    def make(seq):
        def mk(i):
            k, sr = seq[i]
            it = pool[k]
            return serve.Request(rid=i, semiring=sr, operands=it["ops"], mem_bytes=it["bytes"][sr], work=it["work"])
        return mk

    mem_budget = 64 << 30
    # capacity: closed loop, everything queued at once
    cap_seq = draw(400, 7)
    srv = serve.Server(serve.GpuExecutor(args.slots), slots=args.slots, max_batch=8, mem_budget=mem_budget,
                       group_work_max=GROUP_WORK_MAX)
    tc0 = time.perf_counter()
    reqs = serve.run_trace(srv, make(cap_seq), [0.0] * len(cap_seq))
    capacity = len(reqs) / (max(r.t_done for r in reqs) - tc0)
    print(f"[bench] capacity {capacity:.1f} req/s", file=sys.stderr, flush=True)

    warm = 200
    n = warm + args.requests
    seq = draw(n, 11)
    lam = 0.8 * capacity
    arrivals = list(np.cumsum(rng.exponential(1.0 / lam, size=n)))
    keep = set(int(x) for x in np.random.default_rng(3).choice(np.arange(warm, n), size=24, replace=False))

    def run(continuous):
        srv = serve.Server(serve.GpuExecutor(args.slots), slots=args.slots, max_batch=8, mem_budget=mem_budget,
                           continuous=continuous, group_work_max=GROUP_WORK_MAX)
        mk = make(seq)

        def mk2(i):
            r = mk(i)
            r.keep = continuous and i in keep
            return r
        t_begin = time.perf_counter()
        rs = serve.run_trace(srv, mk2, arrivals, timeout=900)
        meas = rs[warm:]
        errs = [r for r in rs if r.error]
        span = max(r.t_done for r in meas) - min(r.t_arrival for r in meas)
        useful = sum(pool[seq[r.rid][0]]["useful"] for r in meas)
        lat = [r.latency * 1e3 for r in meas]
        pc = serve.percentiles(lat)
        return rs, {"requests": len(meas), "errors": len(errs), "throughput_req_s": round(len(meas) / span, 2),
                    "useful_gflops": round(2 * useful / span / 1e9, 3), "p50_ms": round(pc["p50"], 3),
                    "p99_ms": round(pc["p99"], 3), "wall_s": round(time.perf_counter() - t_begin, 2)}

    rs_c, cont = run(True)
    print(f"[bench] continuous {cont}", file=sys.stderr, flush=True)
    _, fifo = run(False)
    print(f"[bench] fifo {fifo}", file=sys.stderr, flush=True)

    # each kept result alone (a fresh single-product run) equals the result in the mix
    same = True
    for r in rs_c:
        if not r.keep or r.error:
            continue
        A, B, M, c = r.operands
        alone = msp.masked_spgemm(A, B, M, complement=c, semiring=r.semiring)
        ok = same_output(r.result.rowptr, r.result.colidx, r.result.values, alone.rowptr, alone.colidx, alone.values,
                         r.semiring == "plus_times_f64")
        same = same and ok
    out = {"metric": "useful_masked_gflops", "value": cont["useful_gflops"], "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.requests, "warmup": warm, "ms_per_step": round(1e3 / cont["throughput_req_s"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "mixed(i64,f64)",
           "data": "synthetic",
           "config": {"workload": "serving: Poisson arrivals at 0.8 x measured capacity over a pool of "
                                  f"{len(pool)} products (Erdos-Renyi n=4096, triangle counting R-MAT 18, BFS "
                                  "step R-MAT 20 x 512 sources, the 64 mixed products at full size), "
                                  "plus-pair int64 / FP64",
                      "slots": args.slots, "max_batch": 8, "group_work_max": GROUP_WORK_MAX,
                      "mem_budget_bytes": mem_budget,
                      "capacity_req_s": round(capacity, 2), "lambda_req_s": round(lam, 2)},
           "serving": {"continuous": cont, "fifo_one_at_a_time": fifo,
                       "speedup_throughput": round(cont["throughput_req_s"] / max(fifo["throughput_req_s"], 1e-9), 3),
                       "alone_equals_mix": same}}
    print(json.dumps(out), flush=True)
    if not same:
        sys.exit(1)


def _counter_kib(csv_dir, counter, kernel_substr):
    """Mean per-dispatch value (KiB) of one counter for the kernels whose name
    contains kernel_substr, from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    vals = []
    for f in glob.glob(os.path.join(csv_dir, "*_counter_collection.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
                    vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} samples for '{kernel_substr}' under {csv_dir}")
    return sum(vals) / len(vals), len(vals)


def summarize_traffic(args):
    """HBM bytes per launch of one kernel from two counter runs, each scaled by
    what the same counter reads for a plain 1 GiB device copy (1 GiB read and
    1 GiB written per launch)."""
    d = args.summarize_traffic
    gib_kib = float(1 << 20)
    cf, _ = _counter_kib(os.path.join(d, "copy_FETCH_SIZE"), "FETCH_SIZE", "copyBuffer")
    cw, _ = _counter_kib(os.path.join(d, "copy_WRITE_SIZE"), "WRITE_SIZE", "copyBuffer")
    key = args.traffic_key
    kf, nf = _counter_kib(os.path.join(d, f"{key}_FETCH_SIZE"), "FETCH_SIZE", args.kernel)
    kw, nw = _counter_kib(os.path.join(d, f"{key}_WRITE_SIZE"), "WRITE_SIZE", args.kernel)
    f_scale, w_scale = gib_kib / cf, gib_kib / cw
    read_b = kf * 1024 * f_scale
    write_b = kw * 1024 * w_scale
    out = {"kernel_hash": kernel_source_hash(), "bin": args.bin, "kernel": args.kernel,
           "hbm_bytes_per_launch": int(round(read_b + write_b)),
           "read_bytes": int(round(read_b)), "write_bytes": int(round(write_b)),
           "fetch_kib_raw": round(kf, 3), "write_kib_raw": round(kw, 3), "dispatches": [nf, nw],
           "copy_fetch_kib_per_gib": round(cf, 3), "copy_write_kib_per_gib": round(cw, 3),
           "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)}
    path = os.path.join(ROOT, "profiles", f"traffic_{key}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def run_copy(args):
    """Calibration for the HBM byte counters: a plain device copy of 1 GiB
    (1 GiB read, 1 GiB written per launch), timed like the other kernels."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    ms = _timed(lambda: dst.copy_(src), args.steps, args.warmup)
    print(json.dumps({"metric": "copy_gbs", "value": round(2 * n / (ms * 1e-3) / 1e9, 1), "unit": "GB/s",
                      "bytes_read": n, "bytes_written": n, "ms_per_copy": round(ms, 4)}), flush=True)


def _timed(fn, steps, warmup, stream=None):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def run_batch(args):
    """64 independent FP64 masked products of uneven sizes (Erdos-Renyi and
    R-MAT, n = 2^U(12,17), degree 2^U(2,6), mask density 10^U(-1,1) times the
    output density; masks at full size unless --mask-cap is given): one batch
    (one launch per kernel bin for all products, replayed from a captured HIP
    graph) against one launch sequence per product on the same GPU, with
    identical outputs, and sampled rows of every product (each product's
    heaviest rows among them) checked against the oracle."""
    import torch

    import mspgen
    import paper_2111_09947_amd as msp
    from paper_2111_09947_amd.autotune import autotune_classes, same_output, table_from_result

    dev = torch.device("cuda:0")
    sr = "plus_times_f64"
    cap = args.mask_cap if args.mask_cap and args.mask_cap > 0 else None
    t0 = time.time()
    prms = mspgen.batch_params(args.batch_count, seed=4)
    devp, host = [], []
    for prm in prms:  # one product at a time: its mask is uploaded and its host copy dropped
        A, B = mspgen.batch_operands(prm)
        M = mspgen.batch_mask(prm, cap)
        devp.append((msp.DeviceCSR.from_host(A, dev, torch.float64), msp.DeviceCSR.from_host(B, dev, torch.float64),
                     msp.DeviceCSR.from_host(M, dev), False))
        host.append(dict(prm=prm, A=A, B=B, mrow=np.diff(M.rowptr)))
        del M
    mask_nnz = int(sum(int(h["mrow"].sum()) for h in host))
    print(f"[bench] batch inputs generated and uploaded ({time.time() - t0:.1f}s): {len(devp)} products, "
          f"{mask_nnz} mask entries", file=sys.stderr, flush=True)
    tune = None
    cfg = {}
    if not args.no_tune:  # the accumulator kind per row class, tuned on this batch
        t1 = time.time()
        tune = autotune_classes(devp, sr, repeats=3)
        cfg = {"kind_table": table_from_result(tune)} if tune["table"] else {}
        print(f"[bench] tuned in {time.time() - t1:.1f}s: {tune['table']} ({tune['default_ms']} -> "
              f"{tune['best_ms']} ms)", file=sys.stderr, flush=True)

    # one launch sequence per product, plans built beforehand
    plans = [msp.Plan(A, B, M, complement=c, semiring=sr, **cfg) for (A, B, M, c) in devp]
    outs = []
    for p, (A, B, M, c) in zip(plans, devp):
        cp = max(p.upper_bound, 1)
        outs.append((torch.empty(A.nrows + 1, dtype=torch.int64, device=dev),
                     torch.empty(cp, dtype=torch.int32, device=dev),
                     torch.empty(cp, dtype=torch.float64, device=dev), cp))

    def per_launch():
        for p, (rp, ci, v, cp) in zip(plans, outs):
            p.execute_into(rp, ci, v, cp)

    ms_single = _timed(per_launch, args.steps, args.warmup)
    print(f"[bench] per-product launches {ms_single:.3f} ms", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    stage_ms = np.zeros(len(msp.STAGE_NAMES))
    with torch.cuda.stream(stream):
        b = msp.Batch(devp, semiring=sr, **cfg)
        b.bind_new_outputs()
        ms_eager = _timed(b.execute, args.steps, args.warmup)
        ms_graph = _timed(b.graph_launch, args.steps, args.warmup)
        timing = msp.Timing(args.steps)
        for _ in range(args.steps):
            b.execute_timed(timing)
        timing.collect(stage_ms)
        timing.close()
        stage_ms /= args.steps
        res = b.results()
        bins = b.row_bins()
    print(f"[bench] batched eager {ms_eager:.3f} ms, graph {ms_graph:.3f} ms", file=sys.stderr, flush=True)

    # identical outputs: batch vs one product at a time
    nnz_single = []
    for p, (rp, ci, v, cp), C in zip(plans, outs, res):
        n = int(rp[-1].item())
        nnz_single.append(n)
        if not same_output(rp, ci[:n], v[:n], C.rowptr, C.colidx, C.values, True):
            print("[bench] MISMATCH between batched and per-product outputs", file=sys.stderr)
            sys.exit(1)
    for p in plans:
        p.close()
    del plans, outs
    torch.cuda.empty_cache()

    # admitted products per row (the plus-pair count), the byte model per row, the sampled oracle check
    import oracle
    with torch.cuda.stream(stream):
        with msp.Batch(devp, semiring="plus_pair_i64") as bp:
            bp.bind_new_outputs()
            bp.execute()
            pair = bp.results()
    per_row, useful = [], 0
    rng = np.random.default_rng(9)
    checked_rows = 0
    t_cpu = 0.0
    cpu_useful = 0
    for h, Cp, C in zip(host, pair, res):
        A, B = h["A"], h["B"]
        prp = Cp.rowptr.cpu().numpy()
        owner = np.repeat(np.arange(A.nrows), np.diff(prp))
        u_row = np.bincount(owner, weights=Cp.values.cpu().numpy(), minlength=A.nrows).astype(np.int64)
        useful += int(u_row.sum())
        fl = row_flops(A, np.diff(B.rowptr))
        rp_h = C.rowptr.cpu().numpy()
        per_row.append(alg_bytes(np.diff(A.rowptr), fl, h["mrow"], u_row, np.diff(rp_h), wA=8, wB=8, wC=8))
        # rows checked against the oracle: a uniform sample plus the heaviest rows by products and by mask length
        rows = np.unique(np.concatenate([rng.integers(0, A.nrows, 16), np.argsort(fl)[-4:],
                                         np.argsort(h["mrow"])[-4:]]))
        Ms = mspgen.batch_mask_rows(h["prm"], rows, cap)
        c0 = time.perf_counter()
        R = oracle.masked_spgemm(A, B, Ms, False, sr, rows=rows)
        t_cpu += time.perf_counter() - c0
        cpu_useful += int(R.useful.sum())
        got = gather_rows(rp_h, C.colidx.cpu().numpy(), C.values.cpu().numpy(), rows)
        if not same_rows(got, (R.rowptr, R.colidx, R.values), True):
            print(f"[bench] MISMATCH against the oracle in product {h['prm']['t']}", file=sys.stderr)
            sys.exit(1)
        checked_rows += len(rows)
    per_row = np.concatenate(per_row)
    products, units, bin_units = int(sum(b.products)), b.units, b.bin_units
    b.close()
    del b, res, pair
    torch.cuda.empty_cache()

    # end to end, planning included
    def single_e2e():
        for (A, B, M, c) in devp:
            with msp.Plan(A, B, M, complement=c, semiring=sr, **cfg) as p:
                p.execute()

    def batch_e2e():
        with torch.cuda.stream(stream):
            with msp.Batch(devp, semiring=sr, **cfg) as bb:
                bb.bind_new_outputs()
                bb.execute()

    e2e_single = _timed(single_e2e, max(1, args.steps // 5), 1)
    e2e_batch = _timed(batch_e2e, max(1, args.steps // 5), 1)

    bin_ms = stage_ms[:len(msp.BIN_NAMES)]
    dom = int(np.argmax(bin_ms))
    dom_bytes = int(per_row[bins == dom].sum())
    achieved = dom_bytes / (bin_ms[dom] * 1e-3) / 1e9 if bin_ms[dom] > 0 else 0.0
    total = int(per_row.sum())
    value = 2 * useful / (ms_graph * 1e-3) / 1e9
    out = {
        "metric": "useful_masked_gflops",
        "value": sig(value),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_graph, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(devp)} FP64 plus-times masked products, Erdos-Renyi / R-MAT mix, "
                               "n 2^12..2^17, degree 4..64, mask 0.1x..10x output density, normal mask",
                   "mask_cap": cap, "mask_nnz": mask_nnz,
                   "rows": int(sum(A.nrows for (A, _, _, _) in devp)), "products": products,
                   "useful_products": useful, "nnz_C": int(sum(nnz_single)), "units": units,
                   "bin_units": bin_units, "kind_table": tune["table"] if tune else None},
        "roofline": {"bound": "hbm", "achieved": sig(achieved), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sig(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"numeric bin {msp.BIN_NAMES[dom]}", "kernel_ms": round(float(bin_ms[dom]), 5),
                     "alg_bytes": dom_bytes},
        "path": {"alg_bytes_total": total,
                 "hbm_frac_whole_step": sig(total / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "stage_ms": {n: round(float(x), 5) for n, x in zip(msp.STAGE_NAMES, stage_ms) if x > 0}},
        "batching": {
            "per_product_launches_ms": round(ms_single, 4),
            "batched_eager_ms": round(ms_eager, 4),
            "batched_graph_ms": round(ms_graph, 4),
            "speedup_graph_vs_per_product": round(ms_single / ms_graph, 3),
            "end_to_end_per_product_ms": round(e2e_single, 3),
            "end_to_end_batched_ms": round(e2e_batch, 3),
            "identical_outputs": True,
        },
        "parity": {"checked": f"{checked_rows} rows over all {len(devp)} products (per product 16 uniform rows and "
                              "its 4 heaviest rows by products and by mask length) against the oracle",
                   "identical_within_tolerance": True},
        "cpu_baseline": {"value": sig(2 * cpu_useful / t_cpu / 1e9), "unit": "GFLOP/s",
                         "cores": oracle.max_threads(), "kind": "oracle",
                         "sample": f"the {checked_rows} checked rows, {t_cpu:.3f} s", "cpu_model": cpu_model()},
        "autotune": tune,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
