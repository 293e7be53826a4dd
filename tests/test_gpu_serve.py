"""Serving loop on the GPU: every request's result in a mixed, continuously
batched run (scenes computed in a batch, or recomputed from a resident
dictionary) equals the oracle's result for its scene, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _pool(seed=4):
    rng = np.random.default_rng(seed)
    pool = []
    for j in range(12):
        ell = int(rng.integers(16, 300))
        n = int(rng.integers(200, 3000))
        pool.append(inputs.planes_in_cube(rng, ell, n))
    pool.append(inputs.clustered_multiset(rng, 100, 64, 5, 100))
    return pool, rng


def _oracle_results(pool):
    out = []
    for R in pool:
        cells, r2c = oracle.dedup(oracle.pack(R, 32), R.shape[1], 32)
        uv, bit, off = oracle.edges(cells, 32)
        out.append({"cells": cells, "row_to_cell": r2c, "uv": uv, "bit": bit, "offsets": off})
    return out


def _check(res, want, rid):
    assert res["status"] == "ok", (rid, res)
    for key in ("cells", "uv", "bit", "offsets", "row_to_cell"):
        assert np.array_equal(res[key], want[key]), (rid, key)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("budget", [None, 0, 200_000])
def test_served_results_equal_oracle(budget):
    """budget None: resident dictionaries within a quarter of free memory
    (every scene becomes resident); 0: none; 200 KB: a few at a time, so the
    LRU evicts while batches are in flight."""
    from paper_1503_06029_amd import serve
    pool, rng = _pool()
    want = _oracle_results(pool)
    t = np.cumsum(rng.exponential(1.0 / 400.0, 150))
    sc = rng.integers(0, len(pool), len(t))
    say("serve", len(t), "requests, resident budget", budget)
    srv = serve.Server(pool, rows_per_class=20000, scenes_per_class=64, resident_budget=budget)
    lat, res, wall = srv.serve(t, sc, keep_results=True)
    assert len(res) == len(t) and (lat > 0).all()
    for rid in range(len(t)):
        _check(res[rid], want[int(sc[rid])], rid)
    nres = sum(1 for r in res.values() if r.get("resident"))
    say("resident results", nres, "pool", None if srv.pool is None else
        (len(srv.pool.scenes), srv.pool.hits, srv.pool.misses, srv.pool.evictions))
    if budget == 0:
        assert srv.pool is None and nres == 0
    else:
        assert nres > 0 and srv.pool.hits == nres
    if budget == 200_000:
        assert srv.pool.evictions > 0 and srv.pool.used <= 200_000


@pytest.mark.timeout(300)
def test_served_cancellation_on_device():
    """Cancelled requests (queued or in flight) are answered "cancelled";
    all others still match the oracle."""
    from paper_1503_06029_amd import serve
    pool, rng = _pool(5)
    want = _oracle_results(pool)
    t = np.cumsum(rng.exponential(1.0 / 400.0, 60))
    sc = rng.integers(0, len(pool), len(t))
    # at arrival (still queued), a few ms later (often in flight), and long after the result
    cancels = [(t[i], i) for i in range(0, len(t), 7)] + [(t[i] + 0.003, i) for i in range(3, len(t), 7)]
    cancels += [(t[-1] + 1.0, len(t) - 1)]
    srv = serve.Server(pool, rows_per_class=20000, scenes_per_class=64)
    lat, res, wall = srv.serve(t, sc, keep_results=True, cancels=cancels)
    assert len(res) == len(t)
    cancelled = set(srv.cancelled)
    assert cancelled <= {i for _, i in cancels} and len(cancelled) > 0
    for rid in range(len(t)):
        if rid in cancelled:
            assert res[rid]["status"] == "cancelled"
        else:
            _check(res[rid], want[int(sc[rid])], rid)
