"""Pins for the CPU oracle (no GPU): brute force on tiny inputs, closed forms,
identities and an independent BFS. Every check is independent of the oracle's
own code path (Gustavson scatter, then mask)."""
import math

import numpy as np
import pytest

import mspgen
import oracle
from tests import brute

SEMIRINGS = ["plus_times_f64", "plus_pair_i64", "lor_land_bool", "plus_times_i32", "plus_times_i64"]
VKIND = {"plus_times_f64": "f64", "plus_pair_i64": "f64", "lor_land_bool": "u8",
         "plus_times_i32": "i32", "plus_times_i64": "i64"}


def _rand_operands(seed, m, k, n, da, db, dm, sr, zeros=True):
    rng = np.random.default_rng(seed)
    A = mspgen.er(m, k, da, seed * 10 + 1, VKIND[sr])
    B = mspgen.er(k, n, db, seed * 10 + 2, VKIND[sr])
    M = mspgen.er(m, n, dm, seed * 10 + 3, "f64")
    if zeros and A.values is not None and A.nnz:
        # explicit stored zeros (and negatives for signed types) must still create entries
        idx = rng.integers(0, A.nnz, size=max(1, A.nnz // 5))
        A.values[idx] = 0
        if sr in ("plus_times_i32", "plus_times_i64") and B.nnz:
            B.values[rng.integers(0, B.nnz, size=max(1, B.nnz // 4))] *= -3
    if M.nnz:
        M.values[:] = 0.0  # mask values are never read: zeros still admit
    return A, B, M


def _norm(v, sr):
    if sr == "plus_times_i32":
        return brute.to_signed(int(v), 32)
    if sr in ("plus_pair_i64", "plus_times_i64"):
        return brute.to_signed(int(v), 64)
    if sr == "lor_land_bool":
        return int(v)
    return v


def _check_sorted(R):
    for s in range(len(R.rowptr) - 1):
        row = R.colidx[R.rowptr[s]:R.rowptr[s + 1]]
        assert np.all(np.diff(row.astype(np.int64)) > 0)


@pytest.mark.parametrize("sr", SEMIRINGS)
@pytest.mark.parametrize("complement", [False, True])
@pytest.mark.parametrize("shape", [(9, 7, 11, 3.0, 2.0, 4.0), (16, 16, 16, 4.0, 4.0, 6.0),
                                   (5, 20, 3, 6.0, 1.0, 1.0), (24, 12, 30, 2.0, 5.0, 12.0)])
def test_oracle_matches_brute_force(sr, complement, shape):
    m, k, n, da, db, dm = shape
    for seed in range(3):
        A, B, M = _rand_operands(seed + 17 * m, m, k, n, da, db, dm, sr)
        R = oracle.masked_spgemm(A, B, M, complement, sr)
        _check_sorted(R)
        got = {key: _norm(v, sr) for key, v in brute.result_dict(R).items()}
        exp = {key: _norm(v, sr) for key, v in brute.brute_masked(A, B, M, complement, sr).items()}
        assert got.keys() == exp.keys()
        for key in exp:
            # same accumulation order (ascending k) -> bit-exact even for f64
            assert got[key] == exp[key], (key, got[key], exp[key])


def test_empty_dimensions():
    for (m, k, n) in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (0, 0, 0)]:
        A = mspgen.er(m, k, 2.0, 1, "f64")
        B = mspgen.er(k, n, 2.0, 2, "f64")
        M = mspgen.er(m, n, 2.0, 3, None)
        for comp in (False, True):
            R = oracle.masked_spgemm(A, B, M, comp, "plus_times_f64")
            assert R.nnz == 0 and len(R.rowptr) == m + 1


def _empty(m, n):
    return mspgen.CSR(m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32))


def _full(m, n):
    r, c = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    return mspgen.from_coo(m, n, r.ravel(), c.ravel())


def _scipy(X):
    import scipy.sparse as sp
    v = np.ones(X.nnz) if X.values is None else X.values.astype(np.float64)
    return sp.csr_matrix((v, X.colidx, X.rowptr), shape=(X.nrows, X.ncols))


def test_mask_special_cases():
    """M empty: normal -> C empty, complement -> plain product; M full:
    normal -> plain product, complement -> empty. The plain product is
    checked against scipy's sparse matrix product (U(0,1) values are
    positive, so no cancellation drops an entry)."""
    A = mspgen.er(40, 30, 4.0, 5, "f64")
    B = mspgen.er(30, 50, 4.0, 6, "f64")
    P = (_scipy(A) @ _scipy(B)).tocsr()
    P.sort_indices()
    for M, comp, expect_plain in [(_empty(40, 50), False, False), (_empty(40, 50), True, True),
                                  (_full(40, 50), False, True), (_full(40, 50), True, False)]:
        R = oracle.masked_spgemm(A, B, M, comp, "plus_times_f64")
        if not expect_plain:
            assert R.nnz == 0
        else:
            assert np.array_equal(R.rowptr, P.indptr)
            assert np.array_equal(R.colidx, P.indices)
            np.testing.assert_allclose(R.values, P.data, rtol=1e-14, atol=0)


@pytest.mark.parametrize("sr", SEMIRINGS)
def test_partition_identity(sr):
    """pattern(C_M) and pattern(C_notM) are disjoint and their union is the
    plain product (complement of an empty mask); values agree entrywise."""
    A, B, M = _rand_operands(3, 50, 40, 60, 5.0, 5.0, 10.0, sr)
    full = brute.result_dict(oracle.masked_spgemm(A, B, _empty(50, 60), True, sr))
    c1 = brute.result_dict(oracle.masked_spgemm(A, B, M, False, sr))
    c2 = brute.result_dict(oracle.masked_spgemm(A, B, M, True, sr))
    assert not (c1.keys() & c2.keys())
    assert (c1.keys() | c2.keys()) == full.keys()
    for key, v in {**c1, **c2}.items():
        assert v == full[key]


def test_identity_operands():
    """A = I gives M .* B exactly; B = I gives M .* A exactly (x * 1.0 is exact)."""
    n = 64
    X = mspgen.er(n, n, 6.0, 9, "f64")
    M = mspgen.er(n, n, 20.0, 10, None)
    I = mspgen.identity(n, "f64")
    Mp = brute.dense_pattern(M)
    for (A, B) in [(I, X), (X, I)]:
        R = oracle.masked_spgemm(A, B, M, False, "plus_times_f64")
        got = brute.result_dict(R)
        exp = {(i, int(X.colidx[p])): X.values[p] for i in range(n)
               for p in range(X.rowptr[i], X.rowptr[i + 1]) if Mp[i, X.colidx[p]]}
        assert got == exp


@pytest.mark.parametrize("sr", ["plus_pair_i64", "plus_times_i32", "lor_land_bool", "plus_times_f64"])
def test_transpose_identity(sr):
    """(M .* (A B))^T = M^T .* (B^T A^T) for commutative (x)."""
    A, B, M = _rand_operands(11, 30, 25, 35, 4.0, 4.0, 8.0, sr)
    for comp in (False, True):
        C = brute.result_dict(oracle.masked_spgemm(A, B, M, comp, sr))
        Ct = brute.result_dict(oracle.masked_spgemm(mspgen.transpose(B), mspgen.transpose(A),
                                                    mspgen.transpose(M), comp, sr))
        assert {(j, i) for (i, j) in C} == set(Ct.keys())
        for (i, j), v in C.items():
            if sr == "plus_times_f64":
                assert abs(Ct[(j, i)] - v) <= 1e-12 * abs(v)
            else:
                assert Ct[(j, i)] == v


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12, 25])
def test_complete_graph_closed_form(n):
    """Triangle counting on K_n: L = strict lower triangle, C = L .* (L L)
    under plus-pair has C(i,j) = i - j - 1 for i - j >= 2 and no other entry;
    nnz(C) = C(n-1, 2) and sum(C) = C(n, 3)."""
    L = mspgen.tril_strict(mspgen.complete_graph(n)) if n > 1 else _empty(n, n)
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    got = brute.result_dict(R)
    exp = {(i, j): i - j - 1 for i in range(n) for j in range(n) if i - j >= 2}
    assert got == exp
    assert R.nnz == math.comb(n - 1, 2) if n >= 3 else R.nnz == 0
    assert int(R.values.sum()) == math.comb(n, 3)


@pytest.mark.parametrize("pq", [(3, 4), (10, 7), (20, 20)])
def test_bipartite_has_no_triangles(pq):
    G = mspgen.complete_bipartite(*pq)
    L = mspgen.tril_strict(mspgen.degree_relabel(G))
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    assert R.nnz == 0


@pytest.mark.parametrize("scale,seed", [(7, 1), (9, 2), (10, 3)])
def test_triangle_count_matches_edge_intersection(scale, seed):
    """sum(L .* (L L)) = trace(A^3)/6, counted independently by neighbour-set
    intersection over edges; the degree relabel must not change it."""
    G = mspgen.rmat_graph(scale, 8, seed)
    expect = brute.triangles_by_intersection(G)
    L = mspgen.tril_strict(mspgen.degree_relabel(G))
    R = oracle.masked_spgemm(L, L, L, False, "plus_pair_i64")
    assert int(R.values.sum()) == expect
    # per-edge support: C(i,j) counts common lower neighbours; total useful = triangles
    assert int(R.useful.sum()) == expect
    L0 = mspgen.tril_strict(G)
    R0 = oracle.masked_spgemm(L0, L0, L0, False, "plus_pair_i64")
    assert int(R0.values.sum()) == expect


def test_int32_wraparound():
    """Path counts above 2^31 wrap mod 2^32 (checked with Python big ints)."""
    k = 1000
    A = mspgen.CSR(1, k, np.array([0, k], np.int64), np.arange(k, dtype=np.int32),
                   np.full(k, 50000, np.int32))
    B = mspgen.CSR(k, 2, np.arange(k + 1, dtype=np.int64), np.zeros(k, np.int32),
                   np.full(k, 47000, np.int32))
    M = _full(1, 2)
    R = oracle.masked_spgemm(A, B, M, False, "plus_times_i32")
    assert R.nnz == 1 and R.colidx[0] == 0
    assert int(R.values[0]) == brute.to_signed(k * 50000 * 47000, 32)
    R64 = oracle.masked_spgemm(A.with_values(A.values.astype(np.int64)),
                               B.with_values(B.values.astype(np.int64)), M, False, "plus_times_i64")
    assert int(R64.values[0]) == k * 50000 * 47000


@pytest.mark.parametrize("sr,vals", [("lor_land_bool", "u8"), ("plus_times_i32", "i32")])
def test_bfs_step_against_queue_bfs(sr, vals):
    """One multi-source BFS step C = !V .* (A F): column s of C holds exactly
    the vertices at distance l_s + 1 from source s; with path-count values
    (plus-times) the entry is the number of shortest paths (Brandes sigma)."""
    G = mspgen.rmat_graph(8, 6, 4)
    F, V, srcs, lv = mspgen.bfs_step_input(G, 24, seed=5, values=vals)
    R = oracle.masked_spgemm(G, F, V, True, sr)
    got = brute.result_dict(R)
    exp = {}
    for s, (src, L) in enumerate(zip(srcs, lv)):
        dist, sigma = brute.bfs_sigma(G, int(src))
        for v, dv in dist.items():
            if dv == L + 1:
                exp[(v, s)] = 1 if sr == "lor_land_bool" else brute.to_signed(sigma[v], 32)
    assert got == exp


def test_useful_product_counter():
    """The oracle's per-row admitted-product count equals the plus-pair sum
    and the dense count sum((A_pat B_pat) .* admitted) computed with numpy."""
    A, B, M = _rand_operands(21, 60, 50, 70, 5.0, 5.0, 15.0, "plus_times_f64")
    Ap = brute.dense_pattern(A).astype(np.int64)
    Bp = brute.dense_pattern(B).astype(np.int64)
    Mp = brute.dense_pattern(M)
    for comp in (False, True):
        adm = Mp != comp
        dense = int(((Ap @ Bp) * adm).sum())
        Rf = oracle.masked_spgemm(A, B, M, comp, "plus_times_f64")
        Rp = oracle.masked_spgemm(A, B, M, comp, "plus_pair_i64")
        assert int(Rf.useful.sum()) == dense == int(Rp.values.sum())


def test_row_subset_matches_full():
    A, B, M = _rand_operands(5, 80, 60, 90, 6.0, 6.0, 12.0, "plus_times_f64")
    full = oracle.masked_spgemm(A, B, M, False, "plus_times_f64")
    rows = np.array([79, 3, 3, 0, 41], np.int64)
    sub = oracle.masked_spgemm(A, B, M, False, "plus_times_f64", rows=rows)
    for s, i in enumerate(rows):
        a = slice(full.rowptr[i], full.rowptr[i + 1])
        b = slice(sub.rowptr[s], sub.rowptr[s + 1])
        assert np.array_equal(full.colidx[a], sub.colidx[b])
        assert np.array_equal(full.values[a], sub.values[b])


def test_dimension_mismatch_rejected():
    A = mspgen.er(5, 6, 2.0, 1, "f64")
    B = mspgen.er(7, 5, 2.0, 2, "f64")
    M = mspgen.er(5, 5, 2.0, 3, None)
    with pytest.raises(ValueError):
        oracle.masked_spgemm(A, B, M, False, "plus_times_f64")


def test_hand_worked_example():
    """tests/golden/hand_example.json: a product worked by hand from the
    definition (both mask modes, plus-times and plus-pair)."""
    from tests.golden_cases import hand_example
    A, B, M, expect = hand_example()
    for key, exp in expect.items():
        sr, mode = key.split("/")
        R = oracle.masked_spgemm(A, B, M, mode == "complement", sr)
        assert R.rowptr.tolist() == exp["rowptr"]
        assert R.colidx.tolist() == exp["colidx"]
        assert R.values.tolist() == exp["values"]
