"""The tree kind of the dictionary: Section 3.2's 2^r-ary tree over the
sorted cells held as index ranges (Algorithm 3's levels), searched digit by
digit for distance-1 queries (Algorithm 4).  Level sizes against Figure 2
and the oracle's level builder; queries against the oracle and the sorted
kind; edges and the fused build unchanged by the kind."""
import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

from conftest import read_golden

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1503_06029_amd import binding, pipeline
    return torch, binding, pipeline


def tree_params(B, r, **kw):
    return B.cg_dict_params_default(kind=B.CG_DICT_TREE, fanout_bits=r, **kw)


def levels_of(g, ell, r):
    """The built dictionary's level sizes (root first), from device memory."""
    depth = (ell + r - 1) // r
    off = g.dict.tree_levels - g.dict_mem.data_ptr()
    return g.dict_mem[off:off + 4 * (depth + 1)].cpu().numpy().view(np.uint32).astype(np.int64)


def test_figure2_levels_and_queries(gpu):
    """Figure 2's six vectors with r = 2: levels 1, 3, 4, 6; every query
    (the vectors, all 64 vectors of length 6) answers as the oracle."""
    torch, B, P = gpu
    g2 = read_golden("fig2.txt")
    vec_rows = [r for r in g2 if r[0] not in ("levels", "path")]
    want_levels = [int(x) for x in next(r for r in g2 if r[0] == "levels")[1:]]
    R = np.array([[int(ch) for ch in r[0]] for r in vec_rows], dtype=np.uint8)
    allq = np.array([[(v >> (5 - i)) & 1 for i in range(6)] for v in range(64)], dtype=np.uint8)
    for wb in (32, 64):
        say("figure 2", wb)
        res = P.cell_graph(R, 6, wb, params=tree_params(B, 2))
        g = res["graph"]
        assert levels_of(g, 6, 2).tolist() == want_levels
        Q = oracle.pack(allq, wb)
        got = g.neighbors_d1(P.to_device_words(Q))
        want = oracle.d1_queries(res["cells"], Q, wb)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("ell,wb,r", [(6, 32, 1), (20, 32, 3), (64, 64, 2), (65, 64, 5), (150, 32, 2),
                                      (150, 64, 8), (300, 64, 7), (1024, 64, 4)])
def test_levels_queries_edges(gpu, ell, wb, r):
    """Clustered sets: level sizes equal the oracle's Algorithm-3 levels;
    queries (cells, random vectors, one-bit flips of cells) equal the
    oracle's; edges equal those of the sorted kind, fused build included."""
    torch, B, P = gpu
    say("tree", ell, wb, r)
    rng = np.random.default_rng(ell * 131 + wb + r)
    R = inputs.clustered_multiset(rng, 150, ell, 5, 40)
    res = P.cell_graph(R, ell, wb, params=tree_params(B, r))
    g = res["graph"]
    cells = res["cells"]
    assert levels_of(g, ell, r).tolist() == oracle.tree_levels(cells, ell, r, wb).tolist()
    Qr = oracle.pack((rng.random((200, ell)) < 0.5).astype(np.uint8), wb)
    bits = np.unpackbits(cells.astype(">u8" if wb == 64 else ">u4").view(np.uint8), axis=1)[:200, :ell]
    Qf = oracle.pack(bits ^ np.eye(ell, dtype=np.uint8)[rng.integers(0, ell, bits.shape[0])], wb)
    for Q in (cells, Qr, Qf):
        got = g.neighbors_d1(P.to_device_words(Q))
        want = oracle.d1_queries(cells, Q, wb)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
    ref = P.cell_graph(R, ell, wb)
    for k in ("ncells", "nedges"):
        assert res[k] == ref[k]
    for k in ("cells", "uv", "bit", "offsets"):
        assert np.array_equal(res[k], ref[k]), k
    # the fused build gives the same levels
    rows = oracle.pack(R, wb)
    gf = P.CellGraph(rows.shape[0], ell, wb, tree_params(B, r))
    gf.dedup_dict(P.to_device_words(rows))
    torch.cuda.synchronize()
    assert levels_of(gf, ell, r).tolist() == levels_of(g, ell, r).tolist()


def test_empty_and_single(gpu):
    """No cells: every level is empty; one cell: one node per level."""
    torch, B, P = gpu
    for n, want in ((0, [0, 0, 0, 0]), (1, [1, 1, 1, 1])):
        R = np.zeros((n, 6), dtype=np.uint8)
        say("tiny", n)
        res = P.cell_graph(R, 6, 64, params=tree_params(B, 2))
        assert levels_of(res["graph"], 6, 2).tolist() == want
