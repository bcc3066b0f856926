"""Builds libmsp.so (the C-ABI library declared in include/msp.h) in-tree
with hipcc for gfx950: every source compiles to its own object in parallel,
then one link."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmsp.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["msp_kernels.hip", "msp_api.hip", "msp_bc.hip", "msp_ktruss.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compiles the library to `out`; `defines` are extra -D options of a
    tuning variant."""
    tag = "_".join(d.replace("=", "-") for d in defines) or "default"
    objdir = os.path.join(OBJDIR, tag)
    os.makedirs(objdir, exist_ok=True)
    dflags = ["-D" + d for d in defines]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        jobs.append((obj, [HIPCC, *FLAGS, *dflags, "-I" + INCLUDE, "-I" + CSRC, "-c", os.path.join(CSRC, s),
                           "-o", obj]))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        rcs = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    if any(rcs):
        raise RuntimeError("hipcc failed compiling libmsp.so")
    tmp = out + ".tmp"
    if _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *(j[0] for j in jobs), "-o", tmp], verbose):
        raise RuntimeError("hipcc failed linking libmsp.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
