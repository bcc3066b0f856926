"""Input generators: determinism, CSR validity and the statistics the
workloads are defined by (statistical checks, not exact pins)."""
import numpy as np

import mspgen


def test_er_deterministic_and_valid():
    a = mspgen.er(500, 400, 8.0, 42, "f64")
    b = mspgen.er(500, 400, 8.0, 42, "f64")
    a.validate()
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.colidx, b.colidx)
    assert np.array_equal(a.values, b.values)
    assert abs(a.nnz / 500 - 8.0) < 0.5
    assert np.all((a.values >= 0) & (a.values < 1))


def test_rmat_graph_shape():
    G = mspgen.rmat_graph(10, 16, 3)
    G.validate()
    assert G.nrows == 1024
    # symmetric, no self loops
    rows = np.repeat(np.arange(G.nrows), np.diff(G.rowptr))
    assert not np.any(rows == G.colidx)
    key = set(zip(rows.tolist(), G.colidx.tolist()))
    assert all((c, r) in key for (r, c) in list(key)[:2000])
    assert G.nnz < 2 * 16 * 1024 and G.nnz > 16 * 1024  # dedup removes a share


def test_relabel_and_tril():
    G = mspgen.rmat_graph(9, 8, 5)
    R = mspgen.degree_relabel(G)
    R.validate()
    deg = np.diff(R.rowptr)
    assert np.all(np.diff(deg) <= 0)
    assert sorted(np.diff(G.rowptr).tolist()) == sorted(deg.tolist())
    L = mspgen.tril_strict(R)
    L.validate()
    rows = np.repeat(np.arange(L.nrows), np.diff(L.rowptr))
    assert np.all(L.colidx < rows)
    assert L.nnz * 2 == R.nnz


def test_bfs_step_input_consistency():
    G = mspgen.rmat_graph(8, 6, 4)
    F, V, srcs, lv = mspgen.bfs_step_input(G, 16, seed=5, values="i32")
    F.validate(); V.validate()
    assert F.ncols == 16 and V.ncols == 16
    Vs = set(zip(np.repeat(np.arange(V.nrows), np.diff(V.rowptr)).tolist(), V.colidx.tolist()))
    Fs = list(zip(np.repeat(np.arange(F.nrows), np.diff(F.rowptr)).tolist(), F.colidx.tolist()))
    assert all(x in Vs for x in Fs)  # the frontier is visited
    assert all((int(s), c) in Vs for c, s in enumerate(srcs))
    assert np.all(F.values >= 1)
    F2, V2, _, _ = mspgen.bfs_step_input(G, 16, seed=5, values="i32")
    assert np.array_equal(F.colidx, F2.colidx) and np.array_equal(V.rowptr, V2.rowptr)


def test_batch_mix_small():
    probs = mspgen.batch_mix(4, seed=4, n_lo=8, n_hi=10)
    assert len(probs) == 4
    for p in probs:
        for X in (p["A"], p["B"], p["M"]):
            X.validate()
        assert p["A"].ncols == p["B"].nrows and p["M"].ncols == p["B"].ncols
        assert 2 ** 8 - 1 <= p["n"] <= 2 ** 10 + 1


def test_er_rows_are_the_rows_of_er():
    """er_rows draws exactly the selected rows of er() (same per-row streams),
    leaving every other row empty."""
    A = mspgen.er(5000, 3000, 40.0, 77, None)
    rows = np.array([0, 17, 4999, 17, 2500])
    S = mspgen.er_rows(5000, 3000, 40.0, 77, rows)
    assert S.nrows == 5000 and S.ncols == 3000
    for i in range(5000):
        exp = A.row(i) if i in (0, 17, 2500, 4999) else np.zeros(0, np.int32)
        assert np.array_equal(S.row(i), exp)


def test_batch_mask_rows_match_the_batch_mask():
    prm = mspgen.batch_params(3, seed=4)[2]
    M = mspgen.batch_mask(prm, max_mask_nnz=300_000)
    rows = np.array([1, 5, prm["n"] - 1])
    S = mspgen.batch_mask_rows(prm, rows, max_mask_nnz=300_000)
    for i in rows:
        assert np.array_equal(S.row(i), M.row(i))
