"""Independent checkers used to pin the oracle (pure Python / numpy, tiny sizes).

None of this shares code with the oracle or with the GPU library.
"""
from __future__ import annotations

from collections import deque

import numpy as np

MASK64 = (1 << 64) - 1
MASK32 = (1 << 32) - 1


def dense_pattern(X):
    P = np.zeros((X.nrows, X.ncols), dtype=bool)
    for i in range(X.nrows):
        P[i, X.colidx[X.rowptr[i]:X.rowptr[i + 1]]] = True
    return P


def dense_values(X, one):
    V = {}
    for i in range(X.nrows):
        for p in range(X.rowptr[i], X.rowptr[i + 1]):
            V[(i, int(X.colidx[p]))] = one if X.values is None else X.values[p]
    return V


def brute_masked(A, B, M, complement, semiring):
    """Per output cell (i, j): admitted = (M has (i,j)) XOR complement; the
    entry exists iff some k has A(i,k) and B(k,j) stored; its value folds the
    products over ascending k (the textbook inner-product definition of a
    matrix product entry, restricted to stored terms).

    Returns dict {(i, j): value} with Python ints (wrapped) or floats."""
    one = {"plus_times_f64": 1.0, "plus_pair_i64": 1, "lor_land_bool": 1,
           "plus_times_i32": 1, "plus_times_i64": 1}[semiring]
    Ap, Bp, Mp = dense_pattern(A), dense_pattern(B), dense_pattern(M)
    Av, Bv = dense_values(A, one), dense_values(B, one)
    out = {}
    for i in range(A.nrows):
        for j in range(B.ncols):
            if bool(Mp[i, j]) == bool(complement):
                continue
            acc = None
            for k in range(A.ncols):
                if not (Ap[i, k] and Bp[k, j]):
                    continue
                a, b = Av[(i, k)], Bv[(k, j)]
                if semiring == "plus_times_f64":
                    t = float(a) * float(b)
                    acc = t if acc is None else acc + t
                elif semiring == "plus_pair_i64":
                    acc = 1 if acc is None else (acc + 1) & MASK64
                elif semiring == "lor_land_bool":
                    t = int(bool(a) and bool(b))
                    acc = t if acc is None else int(bool(acc) or bool(t))
                elif semiring == "plus_times_i32":
                    t = (int(a) * int(b)) & MASK32
                    acc = t if acc is None else (acc + t) & MASK32
                elif semiring == "plus_times_i64":
                    t = (int(a) * int(b)) & MASK64
                    acc = t if acc is None else (acc + t) & MASK64
            if acc is not None:
                out[(i, j)] = acc
    return out


def to_signed(v, bits):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >> (bits - 1) else v


def result_dict(R, rows=None):
    """{(i, j): value} from an oracle/GPU CSR result (rows = row ids of the
    result's rows, default 0..nrows-1)."""
    d = {}
    rows = range(len(R.rowptr) - 1) if rows is None else rows
    for s, i in enumerate(rows):
        for p in range(R.rowptr[s], R.rowptr[s + 1]):
            v = R.values[p]
            d[(int(i), int(R.colidx[p]))] = v.item() if hasattr(v, "item") else v
    return d


def triangles_by_intersection(G):
    """trace(A^3)/6 for a simple undirected graph: every edge (u, v) with
    u < v contributes |N(u) ∩ N(v)|; each triangle is counted on its 3 edges."""
    nbr = [set(G.colidx[G.rowptr[i]:G.rowptr[i + 1]].tolist()) for i in range(G.nrows)]
    total = 0
    for u in range(G.nrows):
        for v in nbr[u]:
            if u < v:
                total += len(nbr[u] & nbr[v])
    assert total % 3 == 0
    return total // 3


def bfs_sigma(G, s):
    """Textbook queue BFS from s with shortest-path counting (Brandes):
    returns (dist, sigma) dicts."""
    dist = {s: 0}
    sigma = {s: 1}
    q = deque([s])
    while q:
        u = q.popleft()
        for p in range(G.rowptr[u], G.rowptr[u + 1]):
            w = int(G.colidx[p])
            if w not in dist:
                dist[w] = dist[u] + 1
                sigma[w] = 0
                q.append(w)
            if dist[w] == dist[u] + 1:
                sigma[w] += sigma[u]
    return dist, sigma
