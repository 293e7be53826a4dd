"""The fused dedup + dictionary build (cg_dedup_dict) against cg_dedup
followed by cg_dict_build: the same cells, row_to_cell, directory and
suffix order, byte for byte, and the same edges; and against the oracle."""
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


def dict_arrays(torch, g):
    """Directory and suffix order of g's dictionary (views into its memory)."""
    d = g.dict
    base = g.dict_mem.data_ptr()
    G = (1 << d.params.dir_bits) + 1
    nc = int(g.ncells.item())
    o_dir, o_sfx = d.dir - base, d.sfx - base
    dir_ = g.dict_mem[o_dir:o_dir + 4 * G].cpu().numpy().view(np.uint32).copy()
    sfx = g.dict_mem[o_sfx:o_sfx + 8 * nc].cpu().numpy().view(np.uint64).copy()
    return dir_, sfx


def both(torch, P, rows, ell, wb, params=None, edge_cap=None):
    from paper_1503_06029_amd import binding as B
    dev = P.to_device_words(rows)
    out = []
    for fused in (False, True):
        g = P.CellGraph(rows.shape[0], ell, wb, params, edge_cap=edge_cap or max(4096, 4 * rows.shape[0]))
        if fused:
            g.dedup_dict(dev)
        else:
            g.dedup(dev)
            g.build_dict()
        g.edges()
        torch.cuda.synchronize()
        res = g.fetch()
        res["dir"], res["sfx"] = dict_arrays(torch, g)
        if g.dict.params.split_bit <= 0 or g.dict.params.path != B.CG_PATH_LOOKUP:
            res["sfx"] = np.zeros(0, np.uint64)  # no suffix order is built (no reader needs it)
        out.append(res)
    return out


def assert_same_build(a, b):
    for k in ("ncells", "nedges", "status"):
        assert a[k] == b[k], k
    for k in ("cells", "row_to_cell", "uv", "bit", "offsets", "dir", "sfx"):
        assert np.array_equal(a[k], b[k]), k


CASES = [("l20", 20, 200, 4, 100, 32), ("l40", 40, 300, 6, 100, 32), ("l64", 64, 300, 6, 100, 64),
         ("l65", 65, 300, 6, 100, 64), ("l130", 130, 700, 10, 700, 64), ("l300", 300, 400, 12, 300, 32),
         ("l1024", 1024, 300, 15, 500, 64),
         # rows of 4, 16, 32 and 64 16-byte pieces: the gather adds a row's
         # suffix-hash terms over that many lanes
         ("l512", 512, 300, 10, 200, 64), ("l2048", 2048, 200, 12, 100, 64),
         ("l4096", 4096, 100, 8, 60, 64), ("l8192", 8192, 60, 6, 40, 64)]


@pytest.mark.parametrize("name,ell,nb,fam,dups,wb", CASES)
def test_fused_equals_separate(gpu, name, ell, nb, fam, dups, wb):
    torch, B, P = gpu
    rng = np.random.default_rng(abs(hash(name)) % (2 ** 32))
    R = inputs.clustered_multiset(rng, nb, ell, fam, dups)
    rows = oracle.pack(R, wb)
    say("fused", name, wb, rows.shape)
    a, b = both(torch, P, rows, ell, wb)
    assert_same_build(a, b)
    cells, r2c = oracle.dedup(rows, ell, wb)
    assert np.array_equal(b["cells"], cells) and np.array_equal(b["row_to_cell"], r2c)


@pytest.mark.parametrize("kw", [dict(split_bit=0, dir_bits=1), dict(split_bit=7, dir_bits=12),
                                dict(split_bit=100, dir_bits=3)])
def test_fused_parameters(gpu, kw):
    torch, B, P = gpu
    rng = np.random.default_rng(5)
    ell = 150
    rows = oracle.pack(inputs.clustered_multiset(rng, 400, ell, 8, 300), 64)
    a, b = both(torch, P, rows, ell, 64, params=B.cg_dict_params_default(**kw))
    assert_same_build(a, b)


def test_fused_heavy_duplicates_and_tiny(gpu):
    torch, B, P = gpu
    rng = np.random.default_rng(9)
    for ell, n, nd in ((70, 20000, 12), (200, 5000, 3), (33, 1, 1), (2000, 3000, 40)):
        rows = oracle.pack(inputs.random_multiset(rng, n, ell, n_distinct=nd), 32)
        say("dups", ell, n, nd)
        a, b = both(torch, P, rows, ell, 32)
        assert_same_build(a, b)


def test_fused_batched_layout(gpu):
    """Tagged virtual rows (scene number in word 0): the directory over the
    tag has long empty stretches (listed gaps)."""
    torch, B, P = gpu
    from paper_1503_06029_amd import batch
    scenes = [inputs.batch_scene(i)[:2000] for i in range(6)]
    sb = batch.SceneBatch([R.shape[1] for R in scenes], [R.shape[0] for R in scenes],
                          batch.class_words(max(R.shape[1] for R in scenes)))
    sb.upload(scenes)
    B.cg_batch_pack(sb.bits, sb.bits_off, sb.scene_ell, sb.scene_rows, sb.n_scenes, sb.n_rows, sb.lay, sb.packed)
    torch.cuda.synchronize()
    rows = sb.packed[:sb.n_rows].cpu().numpy().view(np.uint32)
    a, b = both(torch, P, rows, sb.lay.ell, 32, params=sb.params)
    assert_same_build(a, b)


def test_fused_long_vectors_full_size(gpu):
    """The long-vector workload (probe picks 32-bit sort keys)."""
    torch, B, P = gpu
    rows = inputs.long_vectors()
    want_cells, want_E = inputs.long_vectors_expected()
    a, b = both(torch, P, rows, 1024, 64, edge_cap=want_E + 1024)
    assert b["ncells"] == want_cells and b["nedges"] == want_E
    assert_same_build(a, b)


def _shared_head(rng, n, ell, head_bits):
    """n random rows of ell bits whose first head_bits bits are all equal, so
    32-bit sort keys leave one segment of every row."""
    R = rng.integers(0, 2, size=(n, ell), dtype=np.uint8)
    R[:, :head_bits] = rng.integers(0, 2, size=head_bits, dtype=np.uint8)
    R[n // 2:] = R[:n - n // 2]  # duplicates
    return R


def _grouped_tails(rng, groups, per, ell, head_bits, tail_from):
    """groups x per rows: all share their first head_bits bits; a group's rows
    share bits up to tail_from and differ only after it (plus duplicates), so
    rows tie on every 64-bit value a sort takes before tail_from."""
    R = rng.integers(0, 2, size=(groups * per, ell), dtype=np.uint8)
    R[:, :head_bits] = rng.integers(0, 2, size=head_bits, dtype=np.uint8)
    for g in range(groups):
        R[g * per:(g + 1) * per, head_bits:tail_from] = rng.integers(0, 2, size=tail_from - head_bits,
                                                                      dtype=np.uint8)
    R = np.concatenate([R, R[rng.integers(0, len(R), len(R) // 5)]])  # duplicate rows
    return R[rng.permutation(len(R))]


@pytest.mark.parametrize("key_bits", [0, 32, 64, 96])
def test_tie_runs_in_long_segments(gpu, key_bits):
    """Segments of 129..8,192 rows (one block each) whose rows tie on the
    next 64 bits too: short tie runs (one thread sorts each), long ones (the
    block sorts them), runs of equal rows; against the oracle."""
    torch, B, P = gpu
    rng = np.random.default_rng(71 + key_bits)
    sets = [(_grouped_tails(rng, 60, 25, 300, 40, 140), 32),    # runs of ~25: thread-sorted
            (_grouped_tails(rng, 3, 700, 300, 40, 160), 64),    # runs of ~700: block-sorted
            (_grouped_tails(rng, 1, 3000, 200, 20, 150), 32),   # one segment of 3,000, one run
            (_grouped_tails(rng, 8, 150, 130, 50, 128), 64)]    # rows differing in the last bits only
    for R, wb in sets:
        rows = oracle.pack(R, wb)
        ell = R.shape[1]
        say("tie runs", key_bits, ell, wb, rows.shape)
        a, b = both(torch, P, rows, ell, wb, params=B.cg_dict_params_default(key_bits=key_bits))
        assert_same_build(a, b)
        cells, r2c = oracle.dedup(rows, ell, wb)
        assert np.array_equal(b["cells"], cells) and np.array_equal(b["row_to_cell"], r2c)
        assert np.array_equal(a["cells"], cells) and np.array_equal(a["row_to_cell"], r2c)


@pytest.mark.parametrize("key_bits", [32, 64, 96])
def test_fused_key_bits(gpu, key_bits):
    """A caller-chosen sort-key width changes no byte: clustered sets, rows
    sharing their first 40 bits (one segment of 3,000 / 20,000 rows under
    32-bit keys: the LDS and global-memory tie-fixes), batch-tagged rows,
    against the unfused build (automatic width) and the oracle."""
    torch, B, P = gpu
    rng = np.random.default_rng(11 + key_bits)
    sets = [(inputs.clustered_multiset(rng, 300, 130, 10, 300), 64),
            (inputs.clustered_multiset(rng, 300, 300, 12, 200), 32),
            (_shared_head(rng, 3000, 200, 40), 64),
            (_shared_head(rng, 20000, 96, 40), 32)]
    for R, wb in sets:
        rows = oracle.pack(R, wb)
        ell = R.shape[1]
        say("key_bits", key_bits, ell, wb, rows.shape)
        a, b = both(torch, P, rows, ell, wb, params=B.cg_dict_params_default(key_bits=key_bits))
        assert_same_build(a, b)
        cells, r2c = oracle.dedup(rows, ell, wb)
        assert np.array_equal(b["cells"], cells) and np.array_equal(b["row_to_cell"], r2c)


@pytest.mark.parametrize("key_bits", [32, 64, 96])
def test_fused_long_vectors_key_bits(gpu, key_bits):
    """The long-vector workload with either key width: same bytes as the
    automatic build (which takes 32 bits here)."""
    torch, B, P = gpu
    rows = inputs.long_vectors()
    want_cells, want_E = inputs.long_vectors_expected()
    say("long vectors, key_bits", key_bits)
    dev = P.to_device_words(rows)
    res = []
    for kb in (0, key_bits):
        g = P.CellGraph(rows.shape[0], 1024, 64, B.cg_dict_params_default(key_bits=kb), edge_cap=want_E + 1024)
        g.dedup_dict(dev)
        g.edges()
        torch.cuda.synchronize()
        r = g.fetch()
        r["dir"], r["sfx"] = dict_arrays(torch, g)
        res.append(r)
        del g
    assert res[1]["ncells"] == want_cells and res[1]["nedges"] == want_E
    assert_same_build(res[0], res[1])
