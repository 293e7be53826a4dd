"""Parity of cg_sample_pack (sampled points -> packed sign vectors, on the
GPU) with the CPU oracle under the stated float64 contract: bit-exact."""
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


def random_planes(rng, ell):
    g = rng.standard_normal((ell, 3))
    a = g / np.linalg.norm(g, axis=1, keepdims=True)
    c = rng.uniform(-0.5, 0.5, ell)
    return np.concatenate([a, c[:, None]], axis=1)


@pytest.mark.parametrize("ell,n", [(1, 1000), (31, 5000), (32, 4097), (33, 3000), (64, 10000), (128, 20000),
                                   (300, 3000), (512, 2000)])
@pytest.mark.parametrize("wb", [32, 64])
def test_sample_pack_parity(gpu, ell, n, wb):
    torch, B, P = gpu
    rng = np.random.default_rng(ell * 7 + wb)
    planes = random_planes(rng, ell)
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    seed, scene = 1503, ell
    say("sample", ell, n, wb)
    want = oracle.pack(oracle.sample_signs(planes, n, seed, scene, box), wb)
    g = P.CellGraph(n, ell, wb)
    g.sample(torch.from_numpy(planes).cuda(), seed, scene, box)
    torch.cuda.synchronize()
    got = g.packed[:n].cpu().numpy().view(want.dtype)
    assert np.array_equal(got, want)


def test_sample_then_path(gpu):
    """Sampled scene straight into the path: cells and edges equal the
    oracle's on the oracle's own signs."""
    torch, B, P = gpu
    rng = np.random.default_rng(3)
    ell, n = 40, 30000
    planes = random_planes(rng, ell)
    box = [-1.0, -2.0, -0.5, 1.0, 2.0, 0.5]
    bits = oracle.sample_signs(planes, n, 77, 3, box)
    cells, r2c, uv, bit, off = oracle.cell_graph(bits, ell, 32)
    g = P.CellGraph(n, ell, 32)
    g.sample(torch.from_numpy(planes).cuda(), 77, 3, box)
    g.run_checked()
    res = g.fetch()
    assert np.array_equal(res["cells"], cells)
    assert np.array_equal(res["row_to_cell"], r2c)
    assert np.array_equal(res["uv"], uv)


def test_sample_edge_cases(gpu):
    torch, B, P = gpu
    ell = 5
    # degenerate planes: a = 0, c = 0 gives 1 everywhere; c > 0 gives 0
    planes = np.array([[0, 0, 0, 0.0], [0, 0, 0, 1e-300], [1, 0, 0, 0.0], [0, 1, 0, 2.0], [0, 0, -1, -2.0]])
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    n = 2000
    want = oracle.pack(oracle.sample_signs(planes, n, 0, 0, box), 32)
    g = P.CellGraph(n, ell, 32)
    g.sample(torch.from_numpy(planes).cuda(), 0, 0, box)
    torch.cuda.synchronize()
    got = g.packed[:n].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    assert np.all(got[:, 0] >> 31 == 1) and np.all((got[:, 0] >> 30) & 1 == 0)
    # a box of zero width: every point is lo
    flat = [0.25, 0.25, 0.25, 0.25, 0.25, 0.25]
    want = oracle.pack(oracle.sample_signs(planes, 100, 9, 9, flat), 32)
    g = P.CellGraph(100, ell, 32)
    g.sample(torch.from_numpy(planes).cuda(), 9, 9, flat)
    torch.cuda.synchronize()
    assert np.array_equal(g.packed[:100].cpu().numpy().view(np.uint32), want)
    assert len(np.unique(want)) == 1
    # invalid box is rejected on the host
    with pytest.raises(B.CellGraphError):
        g.sample(torch.from_numpy(planes).cuda(), 0, 0, [1.0, 0, 0, 0.0, 1, 1])


def test_batch_sample_pack_parity(gpu):
    """Many scenes in one launch: each scene's rows equal its oracle signs
    (tag word, then the packed vector), and equal cg_sample_pack's."""
    torch, B, P = gpu
    rng = np.random.default_rng(17)
    ells = [16, 33, 64, 100, 31, 1, 70]
    ns = [500, 1, 0, 2000, 777, 40, 1500]
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    lay = B.cg_batch_layout(max(ells))
    planes = [random_planes(rng, l) for l in ells]
    pool = np.concatenate(planes)
    off = np.concatenate([[0], np.cumsum(ells)[:-1]]).astype(np.int64)
    rows = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    keys = np.array([[1503 + j, 7 * j] for j in range(len(ells))], dtype=np.uint64)
    N = int(rows[-1])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = torch.full((N, lay.words), -1, dtype=torch.int32, device="cuda")
    B.cg_batch_sample_pack(d(pool), d(off), d(np.array(ells, dtype=np.int32)), d(rows), d(keys.view(np.int64)),
                           len(ells), N, box, lay, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    for j, (l, n) in enumerate(zip(ells, ns)):
        say("scene", j, l, n)
        seg = got[rows[j]:rows[j + 1]]
        assert np.all(seg[:, 0] == (j << 16 | j))
        signs = oracle.sample_signs(planes[j], n, int(keys[j, 0]), int(keys[j, 1]), box)
        want = oracle.pack(signs, 32) if n else np.zeros((0, -(-l // 32)), dtype=np.uint32)
        wpad = np.zeros((n, lay.words - 1), dtype=np.uint32)
        wpad[:, :want.shape[1]] = want
        assert np.array_equal(seg[:, 1:], wpad)


def test_sampled_server_matches_single_scenes(gpu):
    """Requests served from scene descriptions (sampled on the GPU in
    batches) give each scene's cells and edges as the oracle computes them
    from the same samples."""
    torch, B, P = gpu
    from paper_1503_06029_amd import serve
    rng = np.random.default_rng(23)
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    descs = []
    for j in range(6):
        l = int(rng.integers(16, 120))
        descs.append((random_planes(rng, l), int(rng.integers(200, 3000)), (99, j)))
    srv = serve.SampledServer(descs, box, rows_per_class=1 << 15, scenes_per_class=64)
    arr = np.sort(rng.uniform(0, 0.02, 30))
    sc = rng.integers(0, len(descs), 30)
    lat, res, wall = srv.serve(arr, sc, keep_results=True)
    want = {}
    for j, (pl, n, key) in enumerate(descs):
        bits = oracle.sample_signs(pl, n, key[0], key[1], box)
        want[j] = oracle.cell_graph(bits, pl.shape[0], 32)
    for rid, si in enumerate(sc):
        cells, r2c, uv, bit, off = want[int(si)]
        r = res[rid]
        assert r["ncells"] == cells.shape[0]
        assert np.array_equal(r["uv"], uv)
        assert np.array_equal(r["row_to_cell"], r2c)
