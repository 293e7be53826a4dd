"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work throughout, so every comparison is bit-exact: packed words,
sorted cells, row_to_cell, cell and edge counts, edge arrays, differing
positions, offsets and distance-1 query masks.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1503_06029_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_digests  # noqa: E402  (reads the committed oracle digests)

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


def oracle_graph(R, ell, wb, packed=False):
    rows = R if packed else oracle.pack(R, wb)
    cells, r2c = oracle.dedup(rows, ell, wb)
    uv, bit, off = oracle.edges(cells, wb)
    return rows, cells, r2c, uv, bit, off


def assert_same(res, ref, check_r2c=True):
    rows, cells, r2c, uv, bit, off = ref
    assert res["ncells"] == cells.shape[0]
    assert np.array_equal(res["cells"], cells)
    if check_r2c:
        assert np.array_equal(res["row_to_cell"], r2c)
    assert res["nedges"] == len(uv)
    assert res["status"] == 0
    assert np.array_equal(res["uv"], uv)
    assert np.array_equal(res["bit"], bit)
    assert np.array_equal(res["offsets"], off)


# ------------------------------------------------------------------- pack

@pytest.mark.parametrize("ell", [1, 5, 16, 31, 32, 33, 63, 64, 65, 100, 128, 257, 1024])
@pytest.mark.parametrize("wb", [32, 64])
def test_pack_parity(gpu, ell, wb):
    torch, B, P = gpu
    say("pack", ell, wb)
    rng = np.random.default_rng(ell * 3 + wb)
    n = 1000
    for stride in (ell, ell + 7, ((ell + 15) // 16) * 16 + 16):
        host = rng.integers(0, 3, (n, stride)).astype(np.uint8)   # values 0/1/2: nonzero is 1
        R = host[:, :ell]
        want = oracle.pack(R, wb)
        bits = torch.from_numpy(host).cuda()
        lay = B.make_layout(ell, wb)
        out = torch.full((n, lay.words), -1, dtype=B.word_dtype(wb), device="cuda")
        B.cg_pack(bits, n, stride, lay, out)
        got = out.cpu().numpy().view(want.dtype)
        assert np.array_equal(got, want), (ell, wb, stride)


# ---------------------------------------------------------- dedup + edges

CASES = [
    # (name, ell, n_bases, fam, dups)
    ("tiny", 3, 4, 2, 5),
    ("l16", 16, 200, 4, 100),
    ("l32", 32, 300, 3, 200),
    ("l63", 63, 300, 6, 100),
    ("l64", 64, 300, 6, 100),
    ("l65", 65, 300, 6, 100),
    ("l100", 100, 500, 8, 400),
    ("l128", 128, 700, 10, 700),
    ("l300", 300, 400, 12, 300),
    ("l1024", 1024, 300, 15, 500),
]


@pytest.mark.parametrize("name,ell,nb,fam,dups", CASES)
@pytest.mark.parametrize("wb", [32, 64])
def test_path_parity_clustered(gpu, name, ell, nb, fam, dups, wb):
    torch, B, P = gpu
    rng = np.random.default_rng(abs(hash((name, wb))) % (2 ** 32))
    R = inputs.clustered_multiset(rng, nb, ell, fam, dups)
    say("clustered", name, wb, R.shape)
    ref = oracle_graph(R, ell, wb)
    res = P.cell_graph(R, ell, wb)
    assert_same(res, ref)


@pytest.mark.parametrize("ell", [7, 20, 40, 70, 200])
def test_dedup_heavy_duplicates(gpu, ell):
    # few distinct rows, many copies: long equal-key segments (the block path)
    torch, B, P = gpu
    rng = np.random.default_rng(ell)
    R = inputs.random_multiset(rng, 20000, ell, n_distinct=12)
    say("heavy-dups", ell)
    for wb in (32, 64):
        ref = oracle_graph(R, ell, wb)
        assert_same(P.cell_graph(R, ell, wb), ref)


def test_dedup_long_shared_prefix(gpu):
    # all rows share their first 64+ bits: one big segment sorted by the tail
    torch, B, P = gpu
    rng = np.random.default_rng(7)
    ell = 200
    R = inputs.clustered_multiset(rng, 300, ell, 4, 300)
    R[:, :120] = 1
    say("shared-prefix", R.shape)
    for wb in (32, 64):
        assert_same(P.cell_graph(R, ell, wb), oracle_graph(R, ell, wb))


@pytest.mark.parametrize("wb", [32, 64])
def test_edge_cases(gpu, wb):
    torch, B, P = gpu
    say("edge cases", wb)
    # empty input
    R = np.zeros((0, 10), dtype=np.uint8)
    res = P.cell_graph(R, 10, wb)
    assert res["ncells"] == 0 and res["nedges"] == 0 and res["offsets"].tolist() == [0]
    # one row; l = 1
    for R, ell in ((np.ones((1, 1), np.uint8), 1), (np.array([[0], [1], [1], [0]], np.uint8), 1),
                   (np.ones((50, 33), np.uint8), 33)):
        assert_same(P.cell_graph(R, ell, wb), oracle_graph(R, ell, wb))
    # full hypercube l = 9 and Figure 1
    n = 2 ** 9
    R = ((np.arange(n)[:, None] >> np.arange(8, -1, -1)[None, :]) & 1).astype(np.uint8)
    R = R[np.random.default_rng(1).permutation(n)]
    res = P.cell_graph(R, 9, wb)
    assert res["nedges"] == 9 * 2 ** 8
    assert_same(res, oracle_graph(R, 9, wb))
    R = np.array([[1, 1, 1], [1, 1, 0], [1, 0, 0], [1, 0, 1]], np.uint8)
    res = P.cell_graph(R, 3, wb)
    assert res["uv"].tolist() == [[0, 1], [0, 2], [1, 3], [2, 3]] and res["bit"].tolist() == [2, 1, 1, 2]


PARAMS = [
    dict(),
    dict(split_bit=0),
    dict(split_bit=1, group_max=1),
    dict(split_bit=7, dir_bits=3, group_max=2),
    dict(split_bit=-1, dir_bits=0, group_max=1024),
    dict(path=1, n_refs=0),
    dict(path=1, n_refs=1),
    dict(path=1, n_refs=4),
    dict(path=1, n_refs=8),
    dict(path=2),
]


@pytest.mark.parametrize("pi", range(len(PARAMS)))
@pytest.mark.parametrize("ell,wb", [(40, 32), (90, 64), (129, 32), (200, 64)])
def test_parameters_do_not_change_bytes(gpu, pi, ell, wb):
    torch, B, P = gpu
    kw = dict(PARAMS[pi])
    if kw.get("split_bit", -1) > ell:
        kw["split_bit"] = ell
    say("params", ell, wb, kw)
    rng = np.random.default_rng(ell + pi)
    R = inputs.clustered_multiset(rng, 250, ell, 6, 100)
    ref = oracle_graph(R, ell, wb)
    params = B.cg_dict_params_default(**kw)
    assert_same(P.cell_graph(R, ell, wb, params=params), ref)


def test_split_at_full_length(gpu):
    torch, B, P = gpu
    rng = np.random.default_rng(3)
    for ell in (20, 64, 100):
        R = inputs.clustered_multiset(rng, 100, ell, 5, 10)
        say("split=l", ell)
        params = B.cg_dict_params_default(split_bit=ell, group_max=3)
        assert_same(P.cell_graph(R, ell, 64, params=params), oracle_graph(R, ell, 64))


# ------------------------------------------------------- capacity overflow

@pytest.mark.parametrize("path", [0, 1, 2])
def test_capacity_overflow(gpu, path):
    torch, B, P = gpu
    say("capacity", path)
    rng = np.random.default_rng(11)
    ell, wb = 70, 64
    R = inputs.clustered_multiset(rng, 100, ell, 5, 50)
    ref = oracle_graph(R, ell, wb)
    E = len(ref[3])
    for cap in (0, 1, E - 1, E):
        g = P.CellGraph(R.shape[0], ell, wb, B.cg_dict_params_default(path=path), edge_cap=cap)
        sentinel = -7
        g.uv.fill_(sentinel)
        g.pack(torch.from_numpy(R).cuda())
        g.run()
        torch.cuda.synchronize()
        assert int(g.nedges.item()) == E
        assert int(g.status.item()) == (B.CG_ECAPACITY if cap < E else B.CG_OK)
        uv = g.uv.cpu().numpy()
        if cap < E:
            assert (uv[cap:] == sentinel).all()  # nothing written at or past cap
        else:
            assert np.array_equal(uv[:E].view(np.uint32), ref[3])
        # regrow and re-run edges only: exact
        g.grow_edges(E)
        g.edges()
        torch.cuda.synchronize()
        assert int(g.status.item()) == B.CG_OK
        assert np.array_equal(g.uv[:E].cpu().numpy().view(np.uint32), ref[3])


# ----------------------------------------------------- distance-1 queries

@pytest.mark.parametrize("ell,wb", [(3, 32), (33, 32), (64, 64), (150, 64), (150, 32), (1024, 64), (4000, 64),
                                    (4000, 32)])
def test_neighbors_d1_parity(gpu, ell, wb):
    torch, B, P = gpu
    say("d1 queries", ell, wb)
    rng = np.random.default_rng(ell * wb)
    R = inputs.clustered_multiset(rng, 200, ell, 6, 50)
    res = P.cell_graph(R, ell, wb)
    g = res["graph"]
    cells = res["cells"]
    # queries: the cells themselves, random vectors, and one-bit flips of cells
    Qr = oracle.pack((rng.random((300, ell)) < 0.5).astype(np.uint8), wb)
    Qf = oracle.pack(np.unpackbits(cells.astype(">u8" if wb == 64 else ">u4").view(np.uint8), axis=1)[:300, :ell]
                     ^ np.eye(ell, dtype=np.uint8)[rng.integers(0, ell, min(300, len(cells)))], wb)
    for Q in (cells, Qr, Qf):
        want = oracle.d1_queries(cells, Q, wb)
        got = g.neighbors_d1(P.to_device_words(Q))
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
    # and with a different directory width
    for p in (0, 1, 5):
        params = B.cg_dict_params_default(dir_bits=min(p, ell))
        g2 = P.cell_graph(R, ell, wb, params=params)["graph"]
        want = oracle.d1_queries(cells, Qr, wb)
        for a, b in zip(g2.neighbors_d1(P.to_device_words(Qr)), want):
            assert np.array_equal(a, b)


# ------------------------------------------------------------ determinism

def test_repeatable_bytes(gpu):
    torch, B, P = gpu
    say("repeat")
    rng = np.random.default_rng(5)
    R = inputs.clustered_multiset(rng, 3000, 256, 10, 3000)
    g = P.CellGraph(R.shape[0], 256, 64)
    bits = torch.from_numpy(R).cuda()
    outs = []
    for _ in range(3):
        g.pack(bits)
        g.run()
        r = g.fetch()
        outs.append((r["cells"].copy(), r["uv"].copy(), r["bit"].copy(), r["row_to_cell"].copy()))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


# -------------------------------------------------------- the workloads

def test_line_arrangement(gpu):
    torch, B, P = gpu
    say("line arrangement")
    R = inputs.line_arrangement()
    ref = oracle_graph(R, 32, 32)
    assert_same(P.cell_graph(R, 32, 32), ref)
    assert_same(P.cell_graph(R, 32, 64), oracle_graph(R, 32, 64))
    for h in (0, 3, 8):
        assert_same(P.cell_graph(R, 32, 32, params=B.cg_dict_params_default(path=B.CG_PATH_ALLPAIRS, n_refs=h)), ref)


@pytest.mark.timeout(600)
def test_plane_arrangement(gpu):
    torch, B, P = gpu
    say("plane arrangement: generate")
    R = inputs.plane_arrangement()
    say("plane arrangement: oracle")
    ref = oracle_graph(R, 128, 32)
    say("plane arrangement: gpu")
    res = P.cell_graph(R, 128, 32)
    assert_same(res, ref)
    assert res["nedges"] <= 1_040_512
    say("plane arrangement: gpu, O(n l) hash path")
    assert_same(P.cell_graph(R, 128, 32, params=B.cg_dict_params_default(path=B.CG_PATH_HASH)), ref)
    for h in (0, 4):
        say("plane arrangement: gpu, (*)-pruned all-pairs, h =", h)
        assert_same(P.cell_graph(R, 128, 32, params=B.cg_dict_params_default(path=B.CG_PATH_ALLPAIRS, n_refs=h)), ref)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.timeout(600)
def test_long_vectors_full_size(gpu):
    """The long-vector workload at its real size, in the launch configuration
    the benchmark times (fused dedup + dictionary build, then cg_edges, edge
    capacity just above the edge count): cells, row_to_cell, edges, bits and
    offsets all equal the oracle's (sort + unique, then Algorithm 4's search
    over the sorted cells), compared through the oracle's committed digests
    (tests/golden/long_vectors_digest.txt, written by make_digests.py)."""
    torch, B, P = gpu
    want = make_digests.read_long()
    say("long vectors: generate")
    rows = inputs.long_vectors()
    assert rows.shape[0] == int(want["rows"][0])
    want_cells, want_E = int(want["cells"][0]), int(want["edges"][0])
    say("long vectors: gpu (bench configuration)")
    g = P.CellGraph(rows.shape[0], 1024, 64, edge_cap=want_E + 1024, with_bits=True)
    dev_rows = P.to_device_words(rows)
    # the benchmark times the key width it measures fastest (32 bits here);
    # the first run takes the automatic width, the second 32 bits
    for kb in (0, 32):
        g.params = B.cg_dict_params_default(key_bits=kb)
        g.dedup_dict(dev_rows)
        g.edges()
        res = g.fetch()
        assert res["ncells"] == want_cells and res["nedges"] == want_E and res["status"] == 0
        say("long vectors: digests")
        assert _sha(res["cells"].astype("<u8")) == want["cells"][1]
        assert _sha(res["row_to_cell"].astype("<u4")) == want["row_to_cell"][0]
        assert _sha(res["uv"].astype("<u4")) == want["uv"][0]
        assert _sha(res["bit"].astype("<u2")) == want["bit"][0]
        assert _sha(res["offsets"].astype("<i8")) == want["offsets"][0]
    # the unfused calls (cg_dedup, cg_dict_build, cg_edges) give the same bytes
    say("long vectors: unfused path")
    res2 = P.cell_graph(rows, 1024, 64, packed=True)
    assert _sha(res2["uv"].astype("<u4")) == want["uv"][0]
    assert _sha(res2["cells"].astype("<u8")) == want["cells"][1]


@pytest.mark.parametrize("i", [0, 1, 2, 3, 5, 8, 13])
def test_batch_scenes(gpu, i):
    torch, B, P = gpu
    ell, n = inputs.batch_scene_params(i)
    if n > 60000:
        pytest.skip("large scene: compared with its oracle digest in test_gpu_full_configs (all 512 scenes)")
    say("batch scene", i, ell, n)
    R = inputs.batch_scene(i)
    wb = 32 if i % 2 else 64
    assert_same(P.cell_graph(R, ell, wb), oracle_graph(R, ell, wb))


@pytest.mark.parametrize("ell,kw", [(10, dict(split_bit=0, group_max=1024)), (12, dict(split_bit=0, group_max=1024)),
                                    (12, dict(split_bit=3)), (12, dict()), (11, dict(split_bit=11, group_max=8)),
                                    (10, dict(split_bit=5)), (10, dict(split_bit=6, group_max=64)),
                                    (9, dict(split_bit=4, group_max=40))])
def test_dense_hypercube_stash_overflow(gpu, ell, kw):
    """Full hypercubes: many edges per tile, so the per-tile edge stashes
    overflow and placement recomputes; long prefix groups take look-ups."""
    torch, B, P = gpu
    say("dense cube", ell, kw)
    n = 2 ** ell
    R = ((np.arange(n)[:, None] >> np.arange(ell - 1, -1, -1)[None, :]) & 1).astype(np.uint8)
    R = R[np.random.default_rng(ell).permutation(n)]
    for wb in (32, 64):
        res = P.cell_graph(R, ell, wb, params=B.cg_dict_params_default(**kw))
        assert res["nedges"] == ell * 2 ** (ell - 1)
        assert_same(res, oracle_graph(R, ell, wb))


def test_wide_rows_generic_paths(gpu):
    """Rows too wide for the LDS tiles (l = 4000): the generic edge passes and
    the large-segment dedup path."""
    torch, B, P = gpu
    rng = np.random.default_rng(21)
    R = inputs.clustered_multiset(rng, 60, 4000, 3, 40)
    say("wide rows", R.shape)
    for wb in (32, 64):
        assert_same(P.cell_graph(R, 4000, wb), oracle_graph(R, 4000, wb))


def test_stash_overflow_past_first_supertile(gpu):
    """A 2^15-cell hypercube as one prefix group: every tile's P stash
    overflows and tiles past the first 64 take their output offset from the
    super-tile totals while most of their threads have nothing to write."""
    torch, B, P = gpu
    ell = 15
    n = 2 ** ell
    R = ((np.arange(n)[:, None] >> np.arange(ell - 1, -1, -1)[None, :]) & 1).astype(np.uint8)
    R = R[np.random.default_rng(15).permutation(n)]
    for wb in (32, 64):
        say("cube 15, split 0", wb)
        res = P.cell_graph(R, ell, wb, params=B.cg_dict_params_default(split_bit=0, group_max=1024))
        assert res["nedges"] == ell * 2 ** (ell - 1)
        assert_same(res, oracle_graph(R, ell, wb))


def test_many_super_tiles(gpu):
    """More than 1,024 super-tiles of capacity (over 16.7M rows): the
    super-tile totals are scanned by their own launch instead of inside each
    placement block.  2^12 cells, each row repeated 4,200 times, packed as
    words: cells are 0 .. 4095 and the edges those of the 12-cube."""
    torch, B, P = gpu
    ell, reps = 12, 4200
    n = (2 ** ell) * reps
    words = np.tile(np.arange(2 ** ell, dtype=np.uint32) << np.uint32(32 - ell), reps)
    words = words[np.random.default_rng(12).permutation(n)].reshape(n, 1)
    say("many super-tiles", n)
    res = P.cell_graph(words, ell, 32, packed=True)
    assert res["ncells"] == 2 ** ell
    cells = (res["cells"][:, 0] >> np.uint32(32 - ell)).astype(np.int64)
    assert np.array_equal(cells, np.arange(2 ** ell))
    assert np.array_equal(res["row_to_cell"], (words[:, 0] >> np.uint32(32 - ell)).astype(np.uint32))
    uv = res["uv"].astype(np.int64)
    assert res["nedges"] == ell * 2 ** (ell - 1)
    x = uv[:, 0] ^ uv[:, 1]
    assert np.all(uv[:, 0] < uv[:, 1]) and np.all((x & (x - 1)) == 0)
    assert np.all(res["bit"] == ell - 1 - np.log2(x).astype(np.int64))
    order = np.lexsort((uv[:, 1], uv[:, 0]))
    assert np.array_equal(order, np.arange(len(uv)))
    deg = np.bincount(uv[:, 0], minlength=2 ** ell)
    assert np.array_equal(res["offsets"], np.concatenate([[0], np.cumsum(deg)]))


def _tie_segments(rng, ell, lens, dup_frac=0.1):
    """Rows in segments that share their first 64 bits.  The first row of
    each segment (placed before the rest, so a stable key sort keeps it
    first) is a base; the others agree with each other on two bit blocks
    where they differ from the base and differ among themselves in a third
    block further on, so they are ordered only by a full-row comparison.
    Every fourth segment uses one-bit flips of the base instead."""
    bases, rest = [], []
    for s, L in enumerate(lens):
        base = rng.integers(0, 2, ell).astype(np.uint8)
        bases.append(base)
        if s % 4 == 3:
            for k in rng.choice(np.arange(64, ell), size=min(L - 1, ell - 64), replace=False):
                r = base.copy()
                r[k] ^= 1
                rest.append(r)
            continue
        a = rng.integers(0, 2, 10).astype(np.uint8)
        b = rng.integers(0, 2, 10).astype(np.uint8)
        for _ in range(L - 1):
            r = base.copy()
            r[100:110] = 1 - base[100:110]
            r[100:110] |= a
            r[300:310] = 1 - base[300:310]
            r[300:310] |= b
            o = int(rng.integers(400, ell - 16))
            r[o:o + 16] = rng.integers(0, 2, 16)
            rest.append(r)
    rest = np.array(rest)
    rest = rest[rng.permutation(len(rest))]
    nd = int(dup_frac * len(rest))
    dups = rest[rng.integers(0, len(rest), nd)]
    return np.concatenate([np.array(bases), rest, dups])


@pytest.mark.parametrize("ell", [600, 2048])
def test_dedup_full_row_ties(gpu, ell):
    """Equal-key segments of 1..300 rows whose order needs full-row
    comparisons, across tile boundaries and around the longest segment the
    summary kernel sorts (128 rows)."""
    torch, B, P = gpu
    rng = np.random.default_rng(ell)
    lens = [1, 2, 3, 17, 64, 127, 128, 129, 300, 2, 5, 128, 40, 1, 129, 77] * 3
    R = _tie_segments(rng, ell, lens)
    for wb in (32, 64):
        say("full-row ties", ell, wb, R.shape)
        rows = oracle.pack(R, wb)
        cells, r2c = oracle.dedup(rows, ell, wb)
        res = P.cell_graph(R, ell, wb)
        assert res["ncells"] == cells.shape[0]
        assert np.array_equal(res["cells"], cells)
        assert np.array_equal(res["row_to_cell"], r2c)


@pytest.mark.parametrize("ell,dup_frac", [(600, 0.0), (600, 0.1), (2048, 0.0)])
def test_dedup_many_short_segments(gpu, ell, dup_frac):
    """Tiles dense with segment heads: 2- and 3-row equal-key segments (up
    to 128 heads in a 256-position tile), beside two long segments."""
    torch, B, P = gpu
    rng = np.random.default_rng(ell + int(100 * dup_frac))
    lens = [2] * 600 + [3] * 200 + [129, 64]
    R = _tie_segments(rng, ell, lens, dup_frac)
    for wb in (32, 64):
        say("short segments", ell, dup_frac, wb, R.shape)
        rows = oracle.pack(R, wb)
        cells, r2c = oracle.dedup(rows, ell, wb)
        res = P.cell_graph(R, ell, wb)
        assert res["ncells"] == cells.shape[0]
        assert np.array_equal(res["cells"], cells)
        assert np.array_equal(res["row_to_cell"], r2c)
