"""The O(n l) edge path (additive-hash probes, one per flip) against the
oracle: the same cells, edges, bits and offsets as the definition gives, on
the shapes the other paths are tested on, and byte-equal to the lookup path."""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1503_06029_amd import binding, pipeline
    return torch, binding, pipeline


def ref_graph(R, ell, wb):
    cells, r2c = oracle.dedup(oracle.pack(R, wb), ell, wb)
    uv, bit, off = oracle.edges(cells, wb)
    return cells, r2c, uv, bit, off


def check(res, ref):
    cells, r2c, uv, bit, off = ref
    assert res["ncells"] == cells.shape[0] and res["nedges"] == len(uv) and res["status"] == 0
    assert np.array_equal(res["cells"], cells)
    assert np.array_equal(res["row_to_cell"], r2c)
    assert np.array_equal(res["uv"], uv)
    assert np.array_equal(res["bit"], bit)
    assert np.array_equal(res["offsets"], off)


def hash_params(B):
    return B.cg_dict_params_default(path=B.CG_PATH_HASH)


@pytest.mark.parametrize("ell", [3, 33, 64, 130, 257, 1024])
@pytest.mark.parametrize("wb", [32, 64])
def test_hash_path_clustered(gpu, ell, wb):
    torch, B, P = gpu
    say("hash path", ell, wb)
    rng = np.random.default_rng(ell * 7 + wb)
    R = inputs.clustered_multiset(rng, 300 if ell < 512 else 80, ell, 8, 400)
    ref = ref_graph(R, ell, wb)
    check(P.cell_graph(R, ell, wb, params=hash_params(B)), ref)
    look = P.cell_graph(R, ell, wb)
    assert np.array_equal(look["uv"], ref[2]) and np.array_equal(look["bit"], ref[3])


@pytest.mark.parametrize("wb", [32, 64])
def test_hash_path_edge_cases(gpu, wb):
    torch, B, P = gpu
    say("hash path edge cases", wb)
    res = P.cell_graph(np.zeros((0, 12), np.uint8), 12, wb, params=hash_params(B))
    assert res["ncells"] == 0 and res["nedges"] == 0 and res["offsets"].tolist() == [0]
    for R, ell in ((np.ones((1, 1), np.uint8), 1), (np.array([[0], [1], [1], [0]], np.uint8), 1),
                   (np.array([[1, 1, 1], [1, 1, 0], [1, 0, 0], [1, 0, 1]], np.uint8), 3)):
        check(P.cell_graph(R, ell, wb, params=hash_params(B)), ref_graph(R, ell, wb))
    # full hypercubes: every cell has l neighbours, l 2^(l-1) edges
    for ell in (9, 12):
        n = 2 ** ell
        R = ((np.arange(n)[:, None] >> np.arange(ell - 1, -1, -1)[None, :]) & 1).astype(np.uint8)
        R = R[np.random.default_rng(ell).permutation(n)]
        res = P.cell_graph(R, ell, wb, params=hash_params(B))
        assert res["nedges"] == ell * 2 ** (ell - 1)
        check(res, ref_graph(R, ell, wb))


def test_hash_path_wide_rows_and_scenes(gpu):
    torch, B, P = gpu
    rng = np.random.default_rng(5)
    R = inputs.clustered_multiset(rng, 40, 4000, 3, 30)
    say("hash path wide rows", R.shape)
    for wb in (32, 64):
        check(P.cell_graph(R, 4000, wb, params=hash_params(B)), ref_graph(R, 4000, wb))
    say("hash path line arrangement")
    R = inputs.line_arrangement()
    check(P.cell_graph(R, 32, 32, params=hash_params(B)), ref_graph(R, 32, 32))
    for i in (0, 3):
        ell, n = inputs.batch_scene_params(i)
        say("hash path batch scene", i, ell, n)
        R = inputs.batch_scene(i)
        check(P.cell_graph(R, ell, 32, params=hash_params(B)), ref_graph(R, ell, 32))
