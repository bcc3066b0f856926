"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU: the
oracle (built with gcc) on small seeded products checked against a dense
brute force, and the C-ABI library's host-side code (its host part built
with the sanitizers, linked with the library's normal device objects) on the
argument, dimension and workspace-size paths that return before any device
work. Each driver exits non-zero on a failed check; a sanitizer finding
aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# sanitizers on the host side only; each -fsanitize= is preceded by -Xarch_host
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, env=None):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr[-4000:]}"
    return res


def test_oracle_under_asan_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "msp_oracle.c"), os.path.join(ROOT, "oracle", "bc_oracle.c"), "-o", exe,
          "-lm"])
    res = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "ok" in res.stdout


def test_abi_host_code_under_asan_ubsan():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    from paper_2111_09947_amd import build as hipbuild
    objdir = os.path.join(hipbuild.OBJDIR, "default")
    others = [os.path.join(objdir, f"{s}.o") for s in ("msp_kernels", "msp_bc", "msp_ktruss")]
    if not all(os.path.exists(o) for o in others):
        hipbuild.build()
    os.makedirs(OUT, exist_ok=True)
    api_o = os.path.join(OUT, "msp_api_san.o")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I" + os.path.join(ROOT, "include"), "-I" + hipbuild.CSRC]
    _run([HIPCC, *common, *HOST_SAN, "-c", os.path.join(hipbuild.CSRC, "msp_api.hip"), "-o", api_o])
    drv_o = os.path.join(OUT, "abi_driver.o")
    _run([HIPCC, *common, *HOST_SAN, "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv_o])
    exe = os.path.join(OUT, "abi_driver")
    _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, drv_o, api_o, *others, "-o", exe])
    # the HIP runtime's own allocations at exit are not this library's: leak checks off
    res = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert "ok" in res.stdout
