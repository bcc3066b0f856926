"""Batched betweenness-centrality dependencies (Section "Betweenness
Centrality": a multi-source forward BFS with a complemented mask, then a
backward dependency sweep with a normal mask).

CPU tests pin the oracle (oracle/bc_oracle.c, Brandes's vertex-by-vertex
recursion) to closed forms and to an independent brute force over pair
dependencies; GPU tests compare the library's matrix formulation
(msp_bc_batch) with the oracle.

Tolerance for the GPU comparison: every dependency is a sum of positive terms
(ratios of path counts times 1 + a positive dependency), so there is no
cancellation; each operation adds at most one rounding of 2^-53 relative, and
a value is built from at most (levels x degree) such operations. 1e-11
relative (plus 1e-9 absolute for values that are 0 on one side only through
rounding) is far above that bound at these sizes and far below any
structural mistake (a missing path changes a value by >= 1/sigma).
"""
import collections
import itertools

import numpy as np
import pytest

import mspgen
import oracle

RTOL = 1e-11


def path_graph(n):
    r = np.arange(n - 1)
    return mspgen.from_coo(n, n, np.concatenate([r, r + 1]), np.concatenate([r + 1, r]))


def star_graph(n):
    leaves = np.arange(1, n)
    return mspgen.from_coo(n, n, np.concatenate([np.zeros(n - 1, int), leaves]),
                           np.concatenate([leaves, np.zeros(n - 1, int)]))


def bfs_all(G, s):
    """Distances and shortest-path counts from s (plain queue BFS)."""
    n = G.nrows
    dist = [-1] * n
    sig = [0] * n
    dist[s], sig[s] = 0, 1
    dq = collections.deque([s])
    while dq:
        u = dq.popleft()
        for w in G.colidx[G.rowptr[u]:G.rowptr[u + 1]]:
            w = int(w)
            if dist[w] < 0:
                dist[w] = dist[u] + 1
                dq.append(w)
            if dist[w] == dist[u] + 1:
                sig[w] += sig[u]
    return dist, sig


def brute_bc(G, sources):
    """Pair-dependency definition: bc[v] = sum_s sum_{t != s, v}
    sigma_st(v) / sigma_st, with sigma_st(v) = sigma_sv * sigma_vt when v
    lies on a shortest s-t path (d_sv + d_vt = d_st); exact fractions."""
    from fractions import Fraction
    n = G.nrows
    info = [bfs_all(G, v) for v in range(n)]
    bc = [Fraction(0)] * n
    for s in sources:
        ds, ss = info[s]
        for v in range(n):
            if v == s or ds[v] < 0:
                continue
            dv, sv = info[v]
            for t in range(n):
                if t in (s, v) or ds[t] < 0:
                    continue
                if ds[v] + dv[t] == ds[t]:
                    bc[v] += Fraction(ss[v] * sv[t], ss[t])
    return np.array([float(x) for x in bc])


# ------------------------------------------------------------ oracle pins

@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_oracle_path_closed_form(n):
    # on a path, the dependency of v on source s is the number of vertices past v, away from s
    G = path_graph(n)
    rng = np.random.default_rng(n)
    src = rng.integers(0, n, size=2 * n)
    v = np.arange(n)
    expect = sum(np.where(v > s, n - 1 - v, np.where(v < s, v, 0)) for s in src).astype(float)
    assert np.array_equal(oracle.bc(G, src), expect)


@pytest.mark.parametrize("n", [3, 9])
def test_oracle_star_and_complete(n):
    bc = oracle.bc(star_graph(n), np.arange(n))
    assert bc[0] == (n - 1) * (n - 2) and np.all(bc[1:] == 0)
    assert np.all(oracle.bc(mspgen.complete_graph(n), np.arange(n)) == 0)


@pytest.mark.parametrize("seed", range(4))
def test_oracle_matches_pair_dependency_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 14
    m = 26
    r = rng.integers(0, n, m)
    c = rng.integers(0, n, m)
    keep = r != c
    G = mspgen.from_coo(n, n, np.concatenate([r[keep], c[keep]]), np.concatenate([c[keep], r[keep]]))
    src = rng.integers(0, n, 6)
    np.testing.assert_allclose(oracle.bc(G, src), brute_bc(G, src), rtol=1e-13, atol=1e-13)


def test_oracle_duplicate_sources_count_twice():
    G = path_graph(6)
    np.testing.assert_array_equal(oracle.bc(G, [2, 2]), 2 * oracle.bc(G, [2]))


# ------------------------------------------------------------ GPU parity

def _bc_gpu(G, src):
    import torch

    import paper_2111_09947_amd as msp
    dev = torch.device("cuda:0")
    dG = msp.DeviceCSR.from_host(G.with_values(None), dev)
    bc, info = msp.bc_batch(dG, np.asarray(src, dtype=np.int32))
    return bc.cpu().numpy(), info


def _close(got, ref):
    np.testing.assert_allclose(got, ref, rtol=RTOL, atol=1e-9)


@pytest.mark.gpu
@pytest.mark.parametrize("n", [2, 7, 20])
def test_gpu_bc_path(n):
    G = path_graph(n)
    src = np.random.default_rng(n).integers(0, n, size=2 * n)
    got, _ = _bc_gpu(G, src)
    _close(got, oracle.bc(G, src))


@pytest.mark.gpu
def test_gpu_bc_star_complete_and_isolated():
    for G, src in [(star_graph(9), np.arange(9)), (mspgen.complete_graph(6), np.arange(6))]:
        got, _ = _bc_gpu(G, src)
        _close(got, oracle.bc(G, src))
    # an isolated source and an edgeless graph give zeros
    G = mspgen.from_coo(5, 5, np.array([0, 1]), np.array([1, 0]))
    got, info = _bc_gpu(G, [3, 4, 0])
    _close(got, oracle.bc(G, [3, 4, 0]))


@pytest.mark.gpu
@pytest.mark.parametrize("scale,nsrc,seed", [(8, 64, 1), (11, 512, 2), (13, 100, 3)])
def test_gpu_bc_rmat(scale, nsrc, seed):
    G = mspgen.rmat_graph(scale, 16, seed)
    deg = np.diff(G.rowptr)
    rng = np.random.default_rng(seed)
    cand = np.nonzero(deg > 0)[0]
    src = rng.choice(cand, size=nsrc, replace=nsrc > len(cand))
    got, info = _bc_gpu(G, src)
    _close(got, oracle.bc(G, src))
    assert info["levels"] >= 1


@pytest.mark.gpu
def test_gpu_bc_duplicate_and_disconnected_sources():
    G = mspgen.rmat_graph(9, 8, 5)
    src = [0, 0, 5, 5, 5, 100, int(np.argmin(np.diff(G.rowptr)))]
    got, _ = _bc_gpu(G, src)
    _close(got, oracle.bc(G, src))
