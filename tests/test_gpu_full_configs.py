"""The batch workload (512 plane scenes) and the served trace over its scene
pool, at their real sizes: every scene's and every request's cells,
row_to_cell, edges, bits and offsets equal the oracle's, compared through
the oracle's committed digests (tests/golden/batch_scenes_digest.txt,
written by tests/golden/make_digests.py from the oracle alone)."""
import hashlib
import os
import sys
import time

import numpy as np
import pytest

from paper_1503_06029_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_digests  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def check_against_digest(r, d, tag):
    assert r["ncells"] == d["ncells"], (tag, "ncells")
    assert r["nedges"] == d["nedges"], (tag, "nedges")
    assert sha(r["cells"].astype("<u4")) == d["cells"], (tag, "cells")
    assert sha(r["row_to_cell"].astype("<u4")) == d["row_to_cell"], (tag, "row_to_cell")
    assert sha(r["uv"].astype("<u4")) == d["uv"], (tag, "uv")
    assert sha(r["bit"].astype("<u2")) == d["bit"], (tag, "bit")
    assert sha(r["offsets"].astype("<i8")) == d["offsets"], (tag, "offsets")


@pytest.fixture(scope="module")
def pool():
    want = make_digests.read_batch()
    assert sorted(want) == list(range(inputs.BATCH_SCENES))
    t0 = time.time()
    scenes = []
    for i in range(inputs.BATCH_SCENES):
        scenes.append(inputs.batch_scene(i))
        if i % 64 == 63:
            say(f"generated {i + 1} scenes, {time.time() - t0:.0f} s")
    for i, R in enumerate(scenes):
        assert R.shape == (want[i]["n"], want[i]["ell"])
    return scenes, want


@pytest.mark.timeout(900)
def test_batch_workload_all_scenes_match_oracle(pool):
    """All 512 scenes in one captured graph (as the benchmark replays it);
    every scene's slice against the oracle's digest, after two replays."""
    import torch
    from paper_1503_06029_amd import batch
    scenes, want = pool
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    say("batch: build runner", sum(n for n, _ in shapes), "rows")
    runner = batch.BatchRunner(shapes, params_for=batch.tuned_params_for())
    runner.upload(scenes)
    runner.run_checked()  # sizes edge buffers
    runner.capture()
    for rep in range(2):
        runner.replay()
        torch.cuda.synchronize()
        say("batch: replay", rep, "fetch")
        res = runner.fetch()
        for i, r in enumerate(res):
            check_against_digest(r, want[i], ("scene", i, "replay", rep))
        say("batch: replay", rep, "all 512 scenes match")


@pytest.mark.timeout(900)
def test_served_trace_every_request_matches_oracle(pool):
    """A served trace over the 512-scene pool (Poisson arrivals at 2,000
    scenes/s): every request's result against the oracle's digest of its
    scene, computed as each result arrives."""
    from paper_1503_06029_amd import serve
    scenes, want = pool
    t, sc = inputs.served_trace(seconds=1.0)
    say("serve:", len(t), "requests")
    srv = serve.Server(scenes)
    seen = {}

    def sink(rid, r):
        assert r["status"] == "ok", (rid, r.get("reason"))
        check_against_digest(r, want[int(sc[rid])], ("request", rid, "scene", int(sc[rid])))
        seen[rid] = True

    lat, _, wall = srv.serve(t, sc, sink=sink)
    assert len(seen) == len(t) and not srv.rejected
    say(f"serve: {len(t)} requests in {wall:.2f} s, p50 {np.percentile(lat, 50) * 1e3:.1f} ms, "
        f"p99 {np.percentile(lat, 99) * 1e3:.1f} ms")
