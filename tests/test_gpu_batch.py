"""Batched scenes (one set of launches for many scenes): every scene's slice
must equal the oracle run on that scene alone, bit for bit, and a captured
HIP graph must give the same bytes on every replay."""
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
    from paper_1503_06029_amd import batch, binding
    return torch, binding, batch


def make_scenes(seed, specs):
    rng = np.random.default_rng(seed)
    scenes = []
    for kind, n, ell in specs:
        if kind == "planes":
            scenes.append(inputs.planes_in_cube(rng, ell, n))
        elif kind == "clustered":
            R = inputs.clustered_multiset(rng, max(1, n // 8), ell, 4, n // 4)
            scenes.append(R)
        else:
            scenes.append((rng.random((n, ell)) < 0.5).astype(np.uint8))
    return scenes


SPECS = [("planes", 2000, 16), ("clustered", 800, 5), ("random", 0, 40), ("random", 1, 33),
         ("planes", 3000, 31), ("clustered", 900, 32), ("planes", 1500, 33), ("clustered", 700, 64),
         ("planes", 2500, 65), ("clustered", 1000, 96), ("planes", 2000, 97), ("clustered", 600, 200),
         ("planes", 1200, 224), ("clustered", 800, 300), ("planes", 1000, 480), ("clustered", 500, 481),
         ("planes", 900, 512), ("random", 300, 7), ("clustered", 400, 128), ("planes", 1800, 150)]


def check_scene(res, R, ell):
    rows = oracle.pack(R, 32)
    cells, r2c = oracle.dedup(rows, ell, 32)
    uv, bit, off = oracle.edges(cells, 32)
    assert res["ncells"] == cells.shape[0]
    assert np.array_equal(res["cells"], cells)
    assert np.array_equal(res["row_to_cell"], r2c)
    assert res["nedges"] == len(uv)
    assert np.array_equal(res["uv"], uv)
    assert np.array_equal(res["bit"], bit)
    assert np.array_equal(res["offsets"], off)


def test_batched_scenes_match_oracle(gpu):
    torch, B, batch = gpu
    scenes = make_scenes(1, SPECS)
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    say("batch", len(scenes), "scenes")
    runner = batch.BatchRunner(shapes)
    runner.upload(scenes)
    runner.run_checked()
    res = runner.fetch()
    for j, (R, r) in enumerate(zip(scenes, res)):
        say("scene", j, R.shape)
        check_scene(r, R, R.shape[1])


def test_batched_graph_replays(gpu):
    torch, B, batch = gpu
    scenes = make_scenes(2, SPECS[:12])
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    say("graph batch", len(scenes))
    runner = batch.BatchRunner(shapes)
    runner.upload(scenes)
    runner.run_checked()  # sizes buffers, warms up
    eager = runner.fetch()
    runner.capture()
    for rep in range(3):
        # clobber the outputs between replays with unrelated eager work
        for _, sb in runner.classes:
            sb.uv.fill_(-1)
            sb.cells.fill_(-1)
            sb.r2c.fill_(-1)
        x = torch.randn(1024, device="cuda").sum()
        torch.cuda.synchronize()
        runner.replay()
        torch.cuda.synchronize()
        got = runner.fetch()
        say("replay", rep, float(x))
        for a, b in zip(got, eager):
            for key in ("cells", "uv", "bit", "offsets", "row_to_cell"):
                assert np.array_equal(a[key], b[key]), (rep, key)
    for j, (R, r) in enumerate(zip(scenes, got)):
        check_scene(r, R, R.shape[1])


def test_tuned_params_keep_bytes(gpu):
    """The autotuner may pick any split / group limit: a tuned class must
    still give the oracle's bytes for every scene."""
    torch, B, batch = gpu
    from paper_1503_06029_amd import tuner
    scenes = make_scenes(3, [s for s in SPECS if 97 <= s[2] <= 224])
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    runner = batch.BatchRunner(shapes)
    runner.upload(scenes)
    tn = tuner.Tuner(path=None)
    for _, sb in runner.classes:
        best, ms = tn.tune_class(sb, reps=1)
        say("tuned", sb.words, best, ms)
    runner.run_checked()
    for j, (R, r) in enumerate(zip(scenes, runner.fetch())):
        check_scene(r, R, R.shape[1])


def test_directory_over_sparse_tags(gpu):
    """Scenes far apart in the tag space leave long empty stretches of the
    prefix directory; d1 queries through it must still find every cell."""
    torch, B, batch = gpu
    scenes = make_scenes(4, [("planes", 1500, 40), ("planes", 900, 60)])
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    runner = batch.BatchRunner(shapes)
    runner.upload(scenes)
    runner.run_checked()
    (_, sb), = runner.classes
    nc = int(sb.ncells.item())
    q = sb.cells[:nc].contiguous()
    self_id = torch.empty(nc, dtype=torch.int32, device="cuda")
    B.cg_neighbors_d1(sb.dict, q, nc, None, self_id, None)
    torch.cuda.synchronize()
    assert np.array_equal(self_id.cpu().numpy(), np.arange(nc, dtype=np.int32))


@pytest.mark.parametrize("shift", [0, 1, 6, 13])
def test_batch_pack_layouts(gpu, shift):
    """cg_batch_pack against the oracle's packing, word for word: the sign
    bytes' base address is `shift` bytes past an aligned one, scenes are
    laid out with gaps between them, and many are tiny or empty (several
    scenes share one block of rows), for every class width."""
    torch, B, batch = gpu
    rng = np.random.default_rng(40 + shift)
    for ell_max in (30, 96, 480, 992):
        ells = [int(rng.integers(1, ell_max + 1)) for _ in range(60)]
        ns = [int(rng.choice([0, 1, 2, 3, 50, 700])) for _ in range(60)]
        ells[0], ns[0] = ell_max, 300
        scenes = [(rng.random((n, l)) < 0.5).astype(np.uint8) for n, l in zip(ns, ells)]
        lay = B.cg_batch_layout(ell_max)
        W = lay.words
        offs, pos = [], 0
        for R in scenes:
            offs.append(pos)
            pos += R.size + int(rng.integers(0, 40))  # gaps between scenes
        host = rng.integers(0, 256, size=shift + pos + 64, dtype=np.uint8)  # garbage around the scenes
        for o, R in zip(offs, scenes):
            host[shift + o:shift + o + R.size] = R.reshape(-1) * rng.integers(1, 256, size=R.size, dtype=np.uint8)
        rows = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        n_rows = int(rows[-1])
        bits = torch.from_numpy(host).cuda()
        packed = torch.empty((max(n_rows, 1), W), dtype=torch.int32, device="cuda")
        say("batch pack", shift, ell_max, W, n_rows)
        B.cg_batch_pack(bits.data_ptr() + shift, torch.tensor(offs, dtype=torch.int64).cuda(),
                        torch.tensor(ells, dtype=torch.int32).cuda(), torch.from_numpy(rows).cuda(), len(scenes),
                        n_rows, lay, packed)
        torch.cuda.synchronize()
        got = packed[:n_rows].cpu().numpy().view(np.uint32)
        want = np.zeros((n_rows, W), np.uint32)
        for j, R in enumerate(scenes):
            if R.shape[0] == 0:
                continue
            want[rows[j]:rows[j + 1], 0] = (j << 16) | j
            p = oracle.pack(R, 32)
            want[rows[j]:rows[j + 1], 1:1 + p.shape[1]] = p
        assert np.array_equal(got, want), (shift, ell_max)
