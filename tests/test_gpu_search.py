"""Parity of the cell-graph search calls (cg_graph_csr, cg_bfs, cg_bfs_path)
with the CPU oracle, through the C ABI.

Adjacency lists, distances and parents are unique (each list ascending; a
parent is the smallest neighbour one level closer), so every comparison is
bit-exact.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

pytestmark = pytest.mark.gpu

NONE = 0xFFFFFFFF


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1503_06029_amd import binding, pipeline
    return torch, binding, pipeline


def grid_bits(k):
    rows = []
    for i in range(k):
        for j in range(k):
            rows.append([1 if i > a else 0 for a in range(k - 1)] + [1 if j > b else 0 for b in range(k - 1)])
    return np.array(rows, dtype=np.uint8)


def graph_of(P, R, ell, wb=64):
    res = P.cell_graph(R, ell, wb)
    return res, res["graph"]


def check_search(torch, B, P, res, g, sources, chunk=64):
    S = P.GraphSearch(g)
    S.build()
    n = res["ncells"]
    uv = res["uv"]
    adj_off, adj = oracle.adjacency(n, uv)
    got = S.fetch()
    assert got["csr_status"] == B.CG_OK
    assert np.array_equal(got["adj_off"], adj_off)
    assert np.array_equal(got["adj"], adj)
    for src in sources:
        say("bfs source", src, "cells", n, "edges", len(uv), "chunk", chunk)
        st = S.bfs_complete(src, chunk)
        assert st == B.CG_OK
        dist, parent, far = oracle.bfs(n, uv, src)
        got = S.fetch()
        assert np.array_equal(got["dist"], dist)
        assert np.array_equal(got["parent"], parent)
        assert got["levels"] == far
    return S


@pytest.mark.parametrize("k", [1, 2, 7, 40])
def test_grid_arrangement(gpu, k):
    torch, B, P = gpu
    R = grid_bits(k) if k > 1 else np.zeros((1, 1), dtype=np.uint8)
    ell = max(2 * (k - 1), 1)
    res, g = graph_of(P, R, ell, 32)
    n = k * k
    S = check_search(torch, B, P, res, g, sorted({0, n - 1, n // 2}))
    # the path to the far corner walks the grid: Manhattan length, one step each
    S.bfs_complete(0)
    p = S.path(n - 1)
    assert len(p) == 2 * (k - 1) + 1 and p[0] == 0 and p[-1] == n - 1
    steps = np.abs(np.diff(p.astype(np.int64)))
    assert np.all((steps == 1) | (steps == k))


@pytest.mark.parametrize("ell", [6, 11])
def test_full_hypercube(gpu, ell):
    torch, B, P = gpu
    n = 2 ** ell
    R = ((np.arange(n)[:, None] >> np.arange(ell - 1, -1, -1)[None, :]) & 1).astype(np.uint8)
    res, g = graph_of(P, R[np.random.default_rng(ell).permutation(n)], ell, 64)
    check_search(torch, B, P, res, g, [0, n - 1, 5])


@pytest.mark.parametrize("name,ell,nb,fam,dups", [("l40", 40, 300, 6, 100), ("l128", 128, 700, 10, 700),
                                                  ("l300", 300, 400, 12, 300)])
def test_clustered_components(gpu, name, ell, nb, fam, dups):
    # many components (one per base family); unreached cells stay unreached
    torch, B, P = gpu
    rng = np.random.default_rng(abs(hash(name)) % (2 ** 32))
    R = inputs.clustered_multiset(rng, nb, ell, fam, dups)
    res, g = graph_of(P, R, ell, 64)
    n = res["ncells"]
    check_search(torch, B, P, res, g, [0, n // 3, n - 1])


def test_plane_arrangement_levels_in_chunks(gpu):
    # an arrangement of planes (the plane-arrangement workload, smaller): one connected graph
    # with many levels, searched one level per call and in chunks of 5
    torch, B, P = gpu
    R = inputs.planes_in_cube(np.random.default_rng(24), 24, 20000)
    res, g = graph_of(P, R, 24, 32)
    n = res["ncells"]
    for chunk in (1, 5):
        check_search(torch, B, P, res, g, [0, n - 1], chunk=chunk)


def test_edge_cases(gpu):
    torch, B, P = gpu
    # one cell, no edges
    R = np.zeros((5, 10), dtype=np.uint8)
    res, g = graph_of(P, R, 10)
    S = check_search(torch, B, P, res, g, [0])
    assert S.fetch()["levels"] == 0
    # source out of range: CG_EINVAL in the status, nothing reached
    S.bfs(3, 4)
    torch.cuda.synchronize()
    assert int(S.status.item()) == B.CG_EINVAL
    assert S.path(0).size == 0
    # isolated cells: only the source is reached
    R = np.array([[0, 0, 0, 0], [1, 1, 0, 0], [0, 0, 1, 1], [1, 1, 1, 1]], dtype=np.uint8)
    res, g = graph_of(P, R, 4)
    assert res["nedges"] == 0
    S = check_search(torch, B, P, res, g, [0, 3])
    d = S.fetch()["dist"]
    assert np.sum(d != NONE) == 1


def test_long_vectors_sampled_sources(gpu):
    """The long-vector workload at full size (4,194,304 cells, 3,932,160
    edges): adjacency against the oracle, and searches from sampled cells
    (each base's star of neighbours is one component)."""
    torch, B, P = gpu
    rows = inputs.long_vectors()
    want_cells, want_E = inputs.long_vectors_expected()
    g = P.CellGraph(rows.shape[0], 1024, 64, edge_cap=want_E + 1024)
    g.run_checked(P.to_device_words(rows))
    nc = int(g.ncells.item())
    uv = g.uv[:int(g.nedges.item())].cpu().numpy().view(np.uint32)
    res = {"ncells": nc, "uv": uv}
    rng = np.random.default_rng(5)
    check_search(torch, B, P, res, g, [int(x) for x in rng.integers(0, nc, 3)])


def test_captured_search_replays(gpu):
    """build() + a full search captured as one graph: every replay (with
    eager work and synchronisation between them) gives the oracle's result."""
    torch, B, P = gpu
    R = inputs.planes_in_cube(np.random.default_rng(31), 32, 30000)
    res, g = graph_of(P, R, 32, 32)
    n = res["ncells"]
    S = P.GraphSearch(g)
    src = n // 2
    S.capture(src, 40)
    dist, parent, far = oracle.bfs(n, res["uv"], src)
    for rep in range(3):
        say("replay", rep)
        S.replay()
        torch.cuda.synchronize()
        got = S.fetch()
        assert got["status"] == B.CG_OK
        assert np.array_equal(got["dist"], dist)
        assert np.array_equal(got["parent"], parent)
        assert got["levels"] == far
        # eager work in between: a search from another cell on the same buffers
        S.bfs_complete(0)
        assert not np.array_equal(S.fetch()["dist"], dist)
