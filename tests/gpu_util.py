"""Helpers shared by the GPU parity tests: upload operands, run the HIP
path through the binding, compare with the oracle (rowptr/colidx exact,
integer values exact, FP64 within 1e-12 relative)."""
import numpy as np
import pytest

import mspgen
import oracle

FP64_RTOL = 1e-12
VKIND = {"plus_times_f64": "f64", "plus_pair_i64": "f64", "lor_land_bool": "u8",
         "plus_times_i32": "i32", "plus_times_i64": "i64"}


def torch_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def msp():
    import paper_2111_09947_amd as m
    return m


def up(X, sr=None):
    torch = torch_or_skip()
    m = msp()
    dt = None if sr is None else m.in_dtype(sr)
    return m.DeviceCSR.from_host(X, torch.device("cuda:0"), dt)


def assert_same(C, R, sr, rows=None):
    """C: DeviceCSR from the GPU; R: oracle result (optionally for `rows`)."""
    rp, ci, v = C.to_host()
    if rows is None:
        assert np.array_equal(rp, R.rowptr), "rowptr differs"
        assert np.array_equal(ci, R.colidx), "colidx differs"
        got = v
    else:
        parts_c, parts_v = [], []
        for i in rows:
            parts_c.append(ci[rp[i]:rp[i + 1]])
            parts_v.append(v[rp[i]:rp[i + 1]])
        lens = np.array([len(p) for p in parts_c])
        assert np.array_equal(lens, np.diff(R.rowptr)), "row lengths differ"
        ci_s = np.concatenate(parts_c) if parts_c else np.zeros(0, np.int32)
        got = np.concatenate(parts_v) if parts_v else np.zeros(0)
        assert np.array_equal(ci_s, R.colidx), "colidx differs"
    exp = R.values
    if sr == "plus_times_f64":
        err = np.abs(got - exp)
        ok = err <= FP64_RTOL * np.abs(exp)
        assert np.all(ok), f"fp64 values differ: max rel {np.max(err / np.maximum(np.abs(exp), 1e-300))}"
    else:
        assert np.array_equal(got, exp), "integer values differ"


def run_and_check(A, B, M, complement, sr, **kw):
    m = msp()
    C = m.masked_spgemm(up(A, sr), up(B, sr), up(M), complement=complement, semiring=sr, **kw)
    R = oracle.masked_spgemm(A, B, M, complement, sr)
    assert_same(C, R, sr)
    return C, R


def rand_problem(seed, m, k, n, da, db, dm, sr):
    A = mspgen.er(m, k, da, seed * 10 + 1, VKIND[sr])
    B = mspgen.er(k, n, db, seed * 10 + 2, VKIND[sr])
    M = mspgen.er(m, n, dm, seed * 10 + 3, None)
    return A, B, M
