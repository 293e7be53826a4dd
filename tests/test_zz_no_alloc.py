"""cg_edges_noalloc (scratch in a static device array, no workspace argument)
against cg_edges with a caller workspace: the same bytes of edges, bits,
offsets, edge count and status, on two calls in a row on one GPU, the second
with a smaller input, and on both edge paths; a call whose scratch need
exceeds the array is refused before anything is launched."""
import os
import sys

import numpy as np
import pytest

from paper_1503_06029_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06029_amd import binding as B
    from paper_1503_06029_amd import pipeline as P
    return torch, B, P


def _both(torch, B, P, R, ell, wb, params=None, cap=None):
    """Build one scene's dictionary, then run cg_edges (workspace) and
    cg_edges_noalloc (static scratch) into separate output buffers."""
    g = P.CellGraph(R.shape[0], ell, wb, params=params, edge_cap=cap)
    bits = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    g.pack(bits)
    g.dedup()
    g.build_dict()
    assert B.cg_edges_workspace(g.dict, g.edge_cap) <= B.NOALLOC_SCRATCH_BYTES
    g.edges()
    dev = g.device
    uv = torch.full_like(g.uv, -1)
    bit = torch.full_like(g.bit, -1)
    off = torch.full_like(g.offsets, -1)
    ne = torch.full((1,), -1, dtype=torch.int64, device=dev)
    st = torch.full((1,), 7, dtype=torch.int32, device=dev)
    B.cg_edges_noalloc(g.dict, uv, bit, g.edge_cap, ne, off, st)
    torch.cuda.synchronize()
    nc = int(g.ncells.item())
    E = int(g.nedges.item())
    assert int(ne.item()) == E
    assert int(st.item()) == int(g.status.item())
    k = min(E, g.edge_cap)
    assert torch.equal(uv[:k], g.uv[:k])
    assert torch.equal(bit[:k], g.bit[:k])
    assert torch.equal(off[:nc + 1], g.offsets[:nc + 1])
    if E > g.edge_cap:  # nothing written at or past the capacity
        assert int(st.item()) == B.CG_ECAPACITY
    return nc, E


@pytest.mark.parametrize("wb", [32, 64])
def test_noalloc_matches_workspace_call_twice(gpu, wb):
    torch, B, P = gpu
    rng = np.random.default_rng(70 + wb)
    big = inputs.clustered_multiset(rng, 400, 200, 12, 6000)   # many tiles, dense groups
    small = inputs.clustered_multiset(rng, 30, 90, 4, 700)      # second call: a smaller input
    say("noalloc", wb, "first call", big.shape)
    nc1, e1 = _both(torch, B, P, big, 200, wb)
    say("noalloc", wb, "second call", small.shape)
    nc2, e2 = _both(torch, B, P, small, 90, wb)
    assert nc2 < nc1 and e1 > 0 and e2 > 0


def test_noalloc_allpairs_path_and_overflow(gpu):
    torch, B, P = gpu
    rng = np.random.default_rng(77)
    R = inputs.clustered_multiset(rng, 60, 140, 6, 1500)
    say("noalloc all-pairs")
    _both(torch, B, P, R, 140, 64, params=B.cg_dict_params_default(path=B.CG_PATH_ALLPAIRS, n_refs=3))
    say("noalloc capacity overflow")
    _both(torch, B, P, R, 140, 32, cap=5)


def test_noalloc_refuses_oversized_scratch(gpu):
    torch, B, P = gpu
    lay = B.make_layout(64, 64)
    n = 4 << 20  # a dictionary over 4M cells needs more edge scratch than the array holds
    cells = torch.zeros((n, 1), dtype=torch.int64, device="cuda")  # full capacity, none of it valid
    ncells = torch.zeros(1, dtype=torch.int64, device="cuda")
    params = B.cg_dict_params_default()
    mem_bytes = B.cg_dict_size(n, lay, params)
    mem = torch.empty(mem_bytes, dtype=torch.uint8, device="cuda")
    d = B.cg_dict_build(cells, ncells, n, lay, params, mem, mem_bytes)
    assert B.cg_edges_workspace(d, 16) > B.NOALLOC_SCRATCH_BYTES
    uv = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    ne = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(B.CellGraphError) as e:
        B.cg_edges_noalloc(d, uv, None, 16, ne, None, st)
    assert e.value.status == B.CG_EWORKSPACE
    torch.cuda.synchronize()
