"""Seeded synthetic inputs for masked sparse products C = M .* (A B).

This module only *builds operands*: Erdos-Renyi and R-MAT graphs, the degree
relabel used before triangle counting, multi-source BFS frontiers, and the
mixed batch of the batched workload. It holds none of the masked-product
arithmetic, and both the CPU oracle (through the tests) and the GPU library
(through the tests and the benchmark) take their inputs from here.

All matrices are returned as :class:`CSR` with int64 row pointers, int32
column indices sorted and duplicate-free within each row, 0-based, and an
optional value array (``None`` means iso-valued: every stored entry is the
semiring's "one").

Workload shapes follow the paper's experimental setup (Section "Experimental
Setup": Erdos-Renyi graphs and R-MAT graphs with Graph500 parameters; the
triangle-counting benchmark relabels vertices by non-increasing degree,
Section "Triangle Counting").
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "CSR", "from_coo", "er", "rmat_edges", "rmat_graph", "degree_relabel",
    "tril_strict", "triangle_input", "bfs_step_input", "batch_mix", "batch_params", "batch_operands",
    "batch_mask", "batch_mask_rows", "er_rows",
    "complete_graph", "complete_bipartite", "identity", "transpose",
    "random_values",
]


@dataclasses.dataclass
class CSR:
    """Host CSR matrix (numpy arrays)."""

    nrows: int
    ncols: int
    rowptr: np.ndarray  # int64 [nrows+1]
    colidx: np.ndarray  # int32 [nnz]
    values: Optional[np.ndarray] = None  # [nnz] or None (iso "one")

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1]) if len(self.rowptr) else 0

    def with_values(self, values: Optional[np.ndarray]) -> "CSR":
        return CSR(self.nrows, self.ncols, self.rowptr, self.colidx, values)

    def row(self, i: int) -> np.ndarray:
        return self.colidx[self.rowptr[i]:self.rowptr[i + 1]]

    def validate(self) -> None:
        rp, ci = self.rowptr, self.colidx
        assert rp.dtype == np.int64 and ci.dtype == np.int32
        assert len(rp) == self.nrows + 1 and rp[0] == 0
        assert np.all(np.diff(rp) >= 0)
        assert len(ci) == rp[-1]
        if len(ci):
            assert ci.min() >= 0 and ci.max() < self.ncols
            # strictly increasing inside each row
            d = np.diff(ci.astype(np.int64))
            starts = np.zeros(len(ci), dtype=bool)
            starts[rp[:-1][rp[:-1] < len(ci)]] = True
            assert np.all((d > 0) | starts[1:])
        if self.values is not None:
            assert len(self.values) == len(ci)


def from_coo(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray,
             values: Optional[np.ndarray] = None, dedup: bool = True) -> CSR:
    """Build a CSR from coordinates; sorts by (row, col). With ``dedup`` the
    first occurrence of a duplicate coordinate is kept."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * np.int64(ncols) + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if dedup and len(key):
        keep = np.ones(len(key), dtype=bool)
        keep[1:] = key[1:] != key[:-1]
        order = order[keep]
        key = key[keep]
    r = key // ncols if ncols else key
    c = key - r * ncols if ncols else key
    counts = np.bincount(r, minlength=nrows) if len(r) else np.zeros(nrows, np.int64)
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    vals = None if values is None else np.asarray(values)[order]
    return CSR(nrows, ncols, rowptr, c.astype(np.int32), vals)


def random_values(nnz: int, kind: Optional[str], rng: np.random.Generator) -> Optional[np.ndarray]:
    """Value arrays per semiring family: 'f64' U(0,1); 'i32' / 'i64' small
    positive integers; 'u8' 0/1 with a few zeros; None -> iso."""
    if kind is None:
        return None
    if kind == "f64":
        return rng.random(nnz)
    if kind == "i32":
        return rng.integers(1, 8, size=nnz, dtype=np.int32)
    if kind == "i64":
        return rng.integers(1, 8, size=nnz, dtype=np.int64)
    if kind == "u8":
        return (rng.random(nnz) < 0.9).astype(np.uint8)
    raise ValueError(kind)


def _er_stream(seed: int, nrows: int, ncols: int, d: float):
    """(numpy generator for the values, 64-bit row-stream seed, p) of er()."""
    rng = np.random.default_rng(seed)
    p = min(1.0, d / ncols) if ncols else 0.0
    if nrows == 0 or ncols == 0:
        return rng, None, p
    return rng, int(rng.integers(0, 2**63 - 1)), p


def er(nrows: int, ncols: int, d: float, seed: int, values: Optional[str] = "f64") -> CSR:
    """Erdos-Renyi G(nrows, ncols, p) with p = d / ncols: every cell is
    present independently, so each row has Binomial(ncols, p) entries at
    distinct uniform columns. Rows are drawn in C by geometric skipping with a
    counter-based random stream per row (mspgen/gen.c); values with numpy."""
    from . import _native
    rng, s64, p = _er_stream(seed, nrows, ncols, d)
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    if s64 is None:
        return CSR(nrows, ncols, rowptr, np.zeros(0, np.int32), random_values(0, values, rng))
    L = _native.lib()
    cnt = np.zeros(nrows, dtype=np.int64)
    L.gen_er_counts(nrows, ncols, p, s64, _native.ptr(cnt))
    np.cumsum(cnt, out=rowptr[1:])
    colidx = np.empty(int(rowptr[-1]), dtype=np.int32)
    L.gen_er_fill(nrows, ncols, p, s64, _native.ptr(rowptr), _native.ptr(colidx))
    return CSR(nrows, ncols, rowptr, colidx, random_values(len(colidx), values, rng))


def er_rows(nrows: int, ncols: int, d: float, seed: int, rows) -> CSR:
    """The rows `rows` of the pattern er(nrows, ncols, d, seed, None) (the same
    per-row random streams), as an nrows x ncols CSR in which every other row
    is empty: enough for an oracle that computes only those rows, without
    drawing the whole matrix."""
    from . import _native
    _, s64, p = _er_stream(seed, nrows, ncols, d)
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    if s64 is None or len(rows) == 0:
        return CSR(nrows, ncols, rowptr, np.zeros(0, np.int32), None)
    L = _native.lib()
    cnt = np.zeros(len(rows), dtype=np.int64)
    L.gen_er_rows_counts(len(rows), _native.ptr(rows), ncols, p, s64, _native.ptr(cnt))
    off = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    colidx = np.empty(int(off[-1]), dtype=np.int32)
    L.gen_er_rows_fill(len(rows), _native.ptr(rows), ncols, p, s64, _native.ptr(off), _native.ptr(colidx))
    full = np.zeros(nrows, dtype=np.int64)
    full[rows] = cnt
    np.cumsum(full, out=rowptr[1:])
    return CSR(nrows, ncols, rowptr, colidx, None)


def rmat_edges(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
               c: float = 0.19) -> Tuple[np.ndarray, np.ndarray]:
    """R-MAT edge list (Graph500 parameters by default): each of
    edge_factor * 2^scale edges picks one of four quadrants per bit level with
    probabilities a, b, c, d = 1 - a - b - c."""
    rng = np.random.default_rng(seed)
    ne = edge_factor << scale
    u = np.zeros(ne, dtype=np.int64)
    v = np.zeros(ne, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for level in range(scale):
        r = rng.random(ne)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        # quadrant: [0,a) -> (0,0); [a,a+b) -> (0,1); [a+b,a+b+c) -> (1,0); else (1,1)
        ubit = r >= ab
        vbit = ((r >= a) & (r < ab)) | (r >= abc)
        u += ubit.astype(np.int64) * bit
        v += vbit.astype(np.int64) * bit
        del r, ubit, vbit
    return u, v


def rmat_graph(scale: int, edge_factor: int, seed: int) -> CSR:
    """Undirected simple graph from R-MAT: drop self loops, symmetrize,
    deduplicate, then apply a seeded random vertex permutation (so that the
    vertex id carries no degree information). Iso-valued pattern."""
    n = 1 << scale
    u, v = rmat_edges(scale, edge_factor, seed)
    keep = u != v
    u, v = u[keep], v[keep]
    perm = np.random.default_rng(seed + 7919).permutation(n).astype(np.int64)
    u, v = perm[u], perm[v]
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    del u, v
    return from_coo(n, n, rows, cols)


def degree_relabel(G: CSR) -> CSR:
    """Relabel vertices in non-increasing degree order; ties keep the old id
    order (stable). Vertex with the largest degree becomes 0."""
    n = G.nrows
    deg = np.diff(G.rowptr)
    order = np.lexsort((np.arange(n), -deg))  # new id -> old id
    newid = np.empty(n, dtype=np.int64)
    newid[order] = np.arange(n, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    return from_coo(n, n, newid[rows], newid[G.colidx.astype(np.int64)], dedup=False)


def tril_strict(G: CSR) -> CSR:
    """Strict lower triangle (j < i) of a square pattern."""
    n = G.nrows
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(G.rowptr))
    cols = G.colidx.astype(np.int64)
    keep = cols < rows
    vals = None if G.values is None else G.values[keep]
    return from_coo(n, G.ncols, rows[keep], cols[keep], vals, dedup=False)


def triangle_input(scale: int, edge_factor: int, seed: int) -> CSR:
    """Triangle counting operand L: R-MAT graph, degree relabel, strict lower
    triangle. Triangle count = sum of L .* (L L) (Section "Triangle
    Counting")."""
    return tril_strict(degree_relabel(rmat_graph(scale, edge_factor, seed)))


def transpose(X: CSR) -> CSR:
    rows = np.repeat(np.arange(X.nrows, dtype=np.int64), np.diff(X.rowptr))
    return from_coo(X.ncols, X.nrows, X.colidx.astype(np.int64), rows, X.values, dedup=False)


def identity(n: int, values: Optional[str] = None) -> CSR:
    v = None if values is None else {"f64": np.ones(n), "i32": np.ones(n, np.int32),
                                     "i64": np.ones(n, np.int64), "u8": np.ones(n, np.uint8)}[values]
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), v)


def complete_graph(n: int) -> CSR:
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = r != c
    return from_coo(n, n, r[keep], c[keep])


def complete_bipartite(p: int, q: int) -> CSR:
    n = p + q
    r, c = np.meshgrid(np.arange(p), np.arange(p, n), indexing="ij")
    rows = np.concatenate([r.ravel(), c.ravel()])
    cols = np.concatenate([c.ravel(), r.ravel()])
    return from_coo(n, n, rows, cols)


def bfs_step_input(G: CSR, nsrc: int, seed: int, values: str = "u8",
                   levels: Optional[List[int]] = None):
    """Operands of one multi-source BFS step in the orientation C = !V .* (A F):
    A = G (n x n, symmetric), F (n x nsrc) holds each source's frontier at its
    depth l_s (values: 1 for 'u8', shortest-path counts for 'i32'/'i64'),
    V (n x nsrc) holds every vertex at distance <= l_s (the visited set).

    Sources are uniform among non-isolated vertices; l_s ~ U{1,2,3}
    (or ``levels`` if given). The per-source BFS runs in C (mspgen/gen.c).
    Returns (F, V, sources, levels)."""
    from . import _native
    rng = np.random.default_rng(seed)
    deg = np.diff(G.rowptr)
    cand = np.nonzero(deg > 0)[0]
    sources = rng.choice(cand, size=nsrc, replace=len(cand) < nsrc).astype(np.int64)
    lv = np.asarray(levels if levels is not None else rng.integers(1, 4, size=nsrc), dtype=np.int32)
    n = G.nrows
    L = _native.lib()
    rp = np.ascontiguousarray(G.rowptr, np.int64)
    ci = np.ascontiguousarray(G.colidx, np.int32)
    fcnt = np.zeros(nsrc, np.int64)
    vcnt = np.zeros(nsrc, np.int64)
    P = _native.ptr
    if L.gen_bfs_counts(n, P(rp), P(ci), nsrc, P(sources), P(lv), P(fcnt), P(vcnt)) != 0:
        raise MemoryError("bfs counts")
    foff = np.zeros(nsrc + 1, np.int64)
    voff = np.zeros(nsrc + 1, np.int64)
    np.cumsum(fcnt, out=foff[1:])
    np.cumsum(vcnt, out=voff[1:])
    fv = np.empty(int(foff[-1]), np.int32)
    fs = np.empty(int(foff[-1]), np.int64)
    vv = np.empty(int(voff[-1]), np.int32)
    if L.gen_bfs_lists(n, P(rp), P(ci), nsrc, P(sources), P(lv), P(foff), P(fv), P(fs), P(voff), P(vv)) != 0:
        raise MemoryError("bfs lists")
    F_rp = np.empty(n + 1, np.int64)
    F_ci = np.empty(len(fv), np.int32)
    F_val = np.empty(len(fv), np.int64)
    L.gen_lists_to_csr(n, nsrc, P(foff), P(fv), P(fs), P(F_rp), P(F_ci), P(F_val))
    del fv, fs
    V_rp = np.empty(n + 1, np.int64)
    V_ci = np.empty(len(vv), np.int32)
    L.gen_lists_to_csr(n, nsrc, P(voff), P(vv), None, P(V_rp), P(V_ci), None)
    if values == "u8":
        fvals = np.ones(len(F_ci), np.uint8)
    elif values == "i32":
        fvals = F_val.astype(np.int32)
    elif values == "i64":
        fvals = F_val
    else:
        fvals = None
    return CSR(n, nsrc, F_rp, F_ci, fvals), CSR(n, nsrc, V_rp, V_ci), sources, lv.astype(np.int64)


def batch_params(count: int, seed: int, n_lo: int = 12, n_hi: int = 17):
    """The drawn parameters of the mixed batch (no matrices): per product
    n = round(2^U(n_lo, n_hi)), input degree d = 2^U(2, 6), mask density
    factor f = 10^U(-1, 1), a sub-seed, and the mask degree
    md = min(n, f * n * (1 - exp(-d^2 / n))), i.e. f times the expected
    Erdos-Renyi density of A B."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(round(2 ** rng.uniform(n_lo, n_hi)))
        d = float(2 ** rng.uniform(2, 6))
        f = float(10 ** rng.uniform(-1, 1))
        sub = int(rng.integers(0, 2**31 - 1))
        dens = 1.0 - math.exp(-d * d / n)
        out.append(dict(t=t, n=n, d=d, f=f, sub=sub, md=min(float(n), f * n * dens)))
    return out


def _mask_degree(prm, max_mask_nnz: Optional[int]) -> float:
    md = prm["md"]
    if max_mask_nnz is not None:
        md = min(md, max_mask_nnz / max(prm["n"], 1))
    return md


def batch_operands(prm):
    """A and B of one product of the mixed batch: Erdos-Renyi for even
    indices, R-MAT (scale round(log2 n), edge factor d / 2, symmetrized)
    truncated to n x n for odd ones; FP64 U(0,1) values."""
    n, d, sub = prm["n"], prm["d"], prm["sub"]
    if prm["t"] % 2 == 0:
        return er(n, n, d, sub + 1, "f64"), er(n, n, d, sub + 2, "f64")
    sc = max(1, int(round(math.log2(n))))
    ef = max(1, int(round(d / 2)))  # each undirected edge appears twice
    G = _truncate(rmat_graph(sc, ef, sub + 3), n)
    vr = np.random.default_rng(sub + 4)
    return G.with_values(vr.random(G.nnz)), G.with_values(vr.random(G.nnz))


def batch_mask(prm, max_mask_nnz: Optional[int] = None) -> CSR:
    """The Erdos-Renyi mask of one product of the mixed batch."""
    n = prm["n"]
    return er(n, n, _mask_degree(prm, max_mask_nnz), prm["sub"] + 5, None)


def batch_mask_rows(prm, rows, max_mask_nnz: Optional[int] = None) -> CSR:
    """Only the rows `rows` of batch_mask(prm) (other rows empty)."""
    n = prm["n"]
    return er_rows(n, n, _mask_degree(prm, max_mask_nnz), prm["sub"] + 5, rows)


def batch_mix(count: int, seed: int, n_lo: int = 12, n_hi: int = 17,
              max_mask_nnz: Optional[int] = None):
    """The mixed batch: ``count`` independent masked products drawn by
    batch_params (Erdos-Renyi or R-MAT A and B, Erdos-Renyi masks, FP64
    U(0,1) values, normal mask).

    ``max_mask_nnz`` caps the mask degree so that reduced-size variants fit a
    CPU check. Returns a list of dicts with A, B, M and the drawn parameters."""
    probs = []
    for prm in batch_params(count, seed, n_lo, n_hi):
        A, B = batch_operands(prm)
        probs.append(dict(A=A, B=B, M=batch_mask(prm, max_mask_nnz), n=prm["n"], d=prm["d"], f=prm["f"]))
    return probs


def _truncate(G: CSR, n: int) -> CSR:
    """Keep the leading n x n block of a square pattern."""
    rows = np.repeat(np.arange(G.nrows, dtype=np.int64), np.diff(G.rowptr))
    cols = G.colidx.astype(np.int64)
    keep = (rows < n) & (cols < n)
    return from_coo(n, n, rows[keep], cols[keep], None, dedup=False)
