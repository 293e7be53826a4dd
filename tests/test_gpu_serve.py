"""Serving loop on the GPU: every request's result in a mixed, continuously
batched run equals the result of that scene computed alone, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(300)
def test_served_results_equal_alone():
    import torch
    from paper_1503_06029_amd import serve, pipeline
    rng = np.random.default_rng(4)
    pool = []
    for j in range(12):
        ell = int(rng.integers(16, 300))
        n = int(rng.integers(200, 3000))
        pool.append(inputs.planes_in_cube(rng, ell, n))
    pool.append(inputs.clustered_multiset(rng, 100, 64, 5, 100))
    t = np.cumsum(rng.exponential(1.0 / 400.0, 150))
    sc = rng.integers(0, len(pool), len(t))
    say("serve", len(t), "requests")
    srv = serve.Server(pool, rows_per_class=20000, scenes_per_class=64)
    lat, res, wall = srv.serve(t, sc, keep_results=True)
    assert len(res) == len(t) and (lat > 0).all()
    alone = {}
    for si, R in enumerate(pool):
        r = pipeline.cell_graph(R, R.shape[1], 32)
        alone[si] = r
    for rid in range(len(t)):
        a, b = res[rid], alone[int(sc[rid])]
        for key in ("cells", "uv", "bit", "offsets", "row_to_cell"):
            assert np.array_equal(a[key], b[key]), (rid, key)
    # and two scenes against the oracle
    for si in (0, len(pool) - 1):
        R = pool[si]
        cells, r2c = oracle.dedup(oracle.pack(R, 32), R.shape[1], 32)
        uv, bit, off = oracle.edges(cells, 32)
        assert np.array_equal(alone[si]["cells"], cells) and np.array_equal(alone[si]["uv"], uv)
