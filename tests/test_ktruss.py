"""k-truss by repeated masked products (Section "Experimental Setup": edges
supported by at least k-2 triangles, the graph shrinking as edges are
pruned). The oracle's iteration is pinned to closed forms and to a plain
edge-peeling brute force; the GPU path (msp_ktruss) is compared with the
oracle bit-exactly (pattern and supports, integer semiring)."""
import itertools

import numpy as np
import pytest

import mspgen
import oracle


def graph(n, edges):
    e = np.array(edges, dtype=np.int64).reshape(-1, 2)
    return mspgen.from_coo(n, n, np.concatenate([e[:, 0], e[:, 1]]), np.concatenate([e[:, 1], e[:, 0]]))


def peel(n, edges, k):
    """Brute force: remove any edge in fewer than k-2 triangles (counted with
    neighbour sets) until none is left to remove; returns {edge: support}."""
    E = {tuple(sorted(e)) for e in edges if e[0] != e[1]}
    while True:
        nb = {v: set() for v in range(n)}
        for a, b in E:
            nb[a].add(b)
            nb[b].add(a)
        sup = {(a, b): len(nb[a] & nb[b]) for a, b in E}
        bad = {e for e, c in sup.items() if c < k - 2}
        if not bad:
            return sup
        E -= bad


def as_dict(rp, ci, sup):
    out = {}
    for i in range(len(rp) - 1):
        for p in range(rp[i], rp[i + 1]):
            out[(i, int(ci[p]))] = int(sup[p])
    return out


def sym(d):
    return {(a, b): c for (a, b), c in d.items()} | {(b, a): c for (a, b), c in d.items()}


@pytest.mark.parametrize("n,k", [(4, 3), (5, 5), (5, 6), (7, 4)])
def test_oracle_complete_graph(n, k):
    rp, ci, sup = oracle.ktruss(mspgen.complete_graph(n), k)
    if k <= n:
        assert len(ci) == n * (n - 1) and np.all(sup == n - 2)
    else:
        assert len(ci) == 0


def test_oracle_diamond_and_pendants():
    # K4 minus an edge: the shared edge is in 2 triangles, the others in 1
    G = graph(5, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4)])
    d3 = as_dict(*oracle.ktruss(G, 3))
    assert d3 == sym({(0, 1): 1, (0, 2): 1, (1, 2): 2, (1, 3): 1, (2, 3): 1})  # the pendant (3,4) goes
    assert len(oracle.ktruss(G, 4)[1]) == 0  # peeling the four outer edges leaves the diagonal unsupported


@pytest.mark.parametrize("seed,k", [(0, 3), (1, 4), (2, 5), (3, 3)])
def test_oracle_matches_edge_peeling(seed, k):
    rng = np.random.default_rng(seed)
    n = 18
    edges = [tuple(e) for e in rng.integers(0, n, size=(70, 2)) if e[0] != e[1]]
    G = graph(n, edges)
    got = as_dict(*oracle.ktruss(G, k))
    assert got == sym(peel(n, edges, k))


def test_oracle_k_at_most_two_returns_graph():
    G = graph(4, [(0, 1), (2, 3)])
    rp, ci, sup = oracle.ktruss(G, 2)
    assert np.array_equal(rp, G.rowptr) and np.array_equal(ci, G.colidx) and np.all(sup == 0)


def _gpu(G, k):
    import torch

    import paper_2111_09947_amd as msp
    dG = msp.DeviceCSR.from_host(G.with_values(None), torch.device("cuda:0"))
    C, info = msp.ktruss(dG, k)
    rp, ci, sup = C.to_host()
    return rp, ci, sup, info


@pytest.mark.gpu
@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
def test_gpu_ktruss_small_graphs(k):
    for G in (mspgen.complete_graph(6), graph(5, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4)]),
              graph(4, [(0, 1)]), graph(3, [])):
        rp, ci, sup, _ = _gpu(G, k)
        erp, eci, esup = oracle.ktruss(G, k)
        assert np.array_equal(rp, erp) and np.array_equal(ci, eci) and np.array_equal(sup, esup)


@pytest.mark.gpu
@pytest.mark.parametrize("scale,k", [(8, 3), (10, 5), (12, 5), (12, 7)])
def test_gpu_ktruss_rmat(scale, k):
    G = mspgen.rmat_graph(scale, 16, scale)
    rp, ci, sup, info = _gpu(G, k)
    erp, eci, esup = oracle.ktruss(G, k)
    assert np.array_equal(rp, erp) and np.array_equal(ci, eci) and np.array_equal(sup, esup)
    assert info["iterations"] >= 1
