"""The resident-dictionary service: membership and distance-1 queries
against device-resident dictionaries, insert-by-rebuild, and the batching
query server, checked against the CPU oracle."""
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
    from paper_1503_06029_amd import binding, pipeline, service
    return torch, binding, pipeline, service


def queries_for(rng, cells, ell, wb, k):
    """Half members, half one-position flips of members (members or not)."""
    q = cells[rng.integers(0, cells.shape[0], k)].copy()
    flip = rng.integers(0, ell, k // 2)
    for r, f in enumerate(flip):
        q[r, f // wb] ^= np.array(1, dtype=q.dtype) << np.array(wb - 1 - f % wb, dtype=q.dtype)
    return q


def check_queries(torch, svc, cells, q, wb):
    d_q = torch.from_numpy(q.view(np.int64 if wb == 64 else np.int32)).cuda()
    m = q.shape[0]
    me = torch.empty(m, dtype=torch.int32, device="cuda")
    cnt = torch.empty(m, dtype=torch.int32, device="cuda")
    mask = torch.empty((m, q.shape[1]), dtype=d_q.dtype, device="cuda")
    svc.query(d_q, me, cnt, mask)
    torch.cuda.synchronize()
    want_cnt, want_self, want_mask = oracle.d1_queries(cells, q, wb)
    assert np.array_equal(me.cpu().numpy().view(np.uint32), want_self)
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32), want_cnt)
    assert np.array_equal(mask.cpu().numpy().view(q.dtype), want_mask)


@pytest.mark.parametrize("ell,wb", [(40, 32), (130, 64), (1024, 64)])
def test_build_query_insert(gpu, ell, wb):
    torch, B, P, S = gpu
    rng = np.random.default_rng(ell + wb)
    R = inputs.clustered_multiset(rng, 300, ell, 8, 200)
    rows = oracle.pack(R, wb)
    half = rows.shape[0] // 2
    svc = S.DictService(ell, wb, capacity=rows.shape[0] + 16)
    dt = np.int64 if wb == 64 else np.int32
    ids = svc.build(torch.from_numpy(rows[:half].view(dt)).cuda())
    cells, r2c = oracle.dedup(rows[:half], ell, wb)
    assert svc.n == cells.shape[0]
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), r2c)
    say("query", ell, wb)
    check_queries(torch, svc, cells, queries_for(rng, cells, ell, wb, 3000), wb)
    # insert the rest: cells of the union, ids of the inserted rows
    new_ids = svc.insert(torch.from_numpy(rows[half:].view(dt)).cuda())
    cells2, _ = oracle.dedup(rows, ell, wb)
    assert svc.n == cells2.shape[0]
    assert np.array_equal(svc.cells[:svc.n].cpu().numpy().view(cells2.dtype), cells2)
    ids2 = new_ids.cpu().numpy().view(np.uint32)
    assert np.array_equal(cells2[ids2], rows[half:])
    check_queries(torch, svc, cells2, queries_for(rng, cells2, ell, wb, 3000), wb)
    # inserting rows that are all present leaves the cells unchanged
    again = svc.insert(torch.from_numpy(rows[:50].view(dt)).cuda())
    assert svc.n == cells2.shape[0]
    assert np.array_equal(cells2[again.cpu().numpy().view(np.uint32)], rows[:50])


def test_query_server_trace(gpu):
    torch, B, P, S = gpu
    rng = np.random.default_rng(11)
    ell, wb = 200, 64
    R = inputs.clustered_multiset(rng, 500, ell, 10, 300)
    rows = oracle.pack(R, wb)
    cells, _ = oracle.dedup(rows, ell, wb)
    svc = S.DictService(ell, wb, capacity=rows.shape[0])
    svc.build(torch.from_numpy(rows.view(np.int64)).cuda())
    reqs = [queries_for(rng, cells, ell, wb, int(k)) for k in rng.integers(1, 200, 300)]
    arr = np.cumsum(rng.exponential(1.0 / 20000, len(reqs)))
    srv = S.QueryServer(svc, max_batch=4096)
    lat, res, wall = srv.serve(arr, reqs)
    assert np.all(lat > 0)
    for q, (me, cnt) in zip(reqs, res):
        want_cnt, want_self, _ = oracle.d1_queries(cells, q, wb)
        assert np.array_equal(me, want_self) and np.array_equal(cnt, want_cnt)
