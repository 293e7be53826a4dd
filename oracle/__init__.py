"""CPU oracle for the cell-graph construction path (arXiv:1503.06029).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_1503_06029_amd``) never imports it and must fail loudly, not fall back
here, when its HIP extension is missing.

Two independent pieces live here:

* ``cg_oracle.c`` -- plain C brute force (pack, sort + unique, all-pairs
  Hamming scan, distance-1 queries, Algorithm 1 distances, the heuristic of
  Algorithm 2 with the corrected filter, the level structure of
  Algorithm 3, and adjacency lists and breadth-first search on the cell
  graph), loaded through ctypes by the thin wrappers below;
* ``twin.py`` -- a pure numpy / Python restatement used to pin the C oracle.

Each C function names the passage of the paper it follows.  Parity status of
every function is listed in the module docstrings; none is unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cg_oracle.c")
# CG_ORACLE_LIB points at another build of cg_oracle.c (the sanitizer test uses it)
_LIB = os.environ.get("CG_ORACLE_LIB") or os.path.join(_HERE, "libcg_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``cg_oracle.c`` into ``libcg_oracle.so`` with gcc + OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-ffp-contract=off",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.cgo_pack.argtypes = [vp, i64, i64, i32, i32, i32, vp]
        L.cgo_pack.restype = i32
        L.cgo_dedup.argtypes = [vp, i64, i32, i32, i32, vp, vp]
        L.cgo_dedup.restype = i64
        L.cgo_dist.argtypes = [vp, vp, i32, i32]
        L.cgo_dist.restype = i64
        L.cgo_dist_bitwise.argtypes = [vp, vp, i32, i32]
        L.cgo_dist_bitwise.restype = i64
        L.cgo_edges.argtypes = [vp, i64, i32, i32, i64, vp, vp, vp, vp]
        L.cgo_edges.restype = i64
        L.cgo_edges_search.argtypes = [vp, i64, i32, i32, i32, i64, vp, vp, vp, vp]
        L.cgo_edges_search.restype = i64
        L.cgo_neighbors_of.argtypes = [vp, i64, i32, i32, vp, i64, i32, vp, vp]
        L.cgo_neighbors_of.restype = i32
        L.cgo_d1_queries.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp, vp]
        L.cgo_d1_queries.restype = i32
        L.cgo_ref_dists.argtypes = [vp, i64, vp, i32, i32, i32, vp]
        L.cgo_ref_dists.restype = i32
        L.cgo_edges_heuristic.argtypes = [vp, i64, i32, i32, vp, i32, i64, vp, vp]
        L.cgo_edges_heuristic.restype = i64
        L.cgo_tree_levels.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp, vp, vp]
        L.cgo_tree_levels.restype = i64
        L.cgo_digits.argtypes = [vp, i32, i32, i32, vp]
        L.cgo_digits.restype = i32
        L.cgo_threads.restype = i32
        L.cgo_set_threads.argtypes = [i32]
        L.cgo_set_threads.restype = None
        L.cgo_adjacency.argtypes = [i64, i64, vp, vp, vp]
        L.cgo_adjacency.restype = i32
        L.cgo_bfs.argtypes = [i64, vp, vp, ctypes.c_uint32, vp, vp]
        L.cgo_bfs.restype = i64
        L.cgo_philox4x64.argtypes = [vp, vp, vp]
        L.cgo_philox4x64.restype = None
        L.cgo_sample_point.argtypes = [i64, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
        L.cgo_sample_point.restype = None
        L.cgo_sample_signs.argtypes = [vp, i32, i64, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
        L.cgo_sample_signs.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _wdtype(word_bits: int):
    if word_bits == 64:
        return np.uint64
    if word_bits == 32:
        return np.uint32
    raise ValueError("word_bits must be 32 or 64")


def words_for(ell: int, word_bits: int) -> int:
    return max(1, -(-ell // word_bits))


def threads() -> int:
    return int(lib().cgo_threads())


def set_threads(n: int) -> None:
    """Threads for the parallel loops from now on (results do not depend on it)."""
    lib().cgo_set_threads(int(n))


def pack(bits: np.ndarray, word_bits: int = 64) -> np.ndarray:
    """O1: uint8 (n, l) sign matrix -> (n, words) packed rows, MSB first."""
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    n, ell = bits.shape
    W = words_for(ell, word_bits)
    out = np.zeros((n, W), dtype=_wdtype(word_bits))
    rc = lib().cgo_pack(_p(bits), n, ell, ell, word_bits, W, _p(out))
    assert rc == 0
    return out


def dedup(rows: np.ndarray, ell: int, word_bits: int = 64):
    """O2: packed rows (n, W) -> (cells (n_cells, W), row_to_cell (n,) uint32)."""
    rows = np.ascontiguousarray(rows)
    n, W = rows.shape
    assert rows.dtype == _wdtype(word_bits)
    cells = np.zeros_like(rows)
    r2c = np.zeros(n, dtype=np.uint32)
    nc = lib().cgo_dedup(_p(rows), n, ell, word_bits, W, _p(cells), _p(r2c))
    assert nc >= 0
    return cells[:nc].copy(), r2c


def edges(cells: np.ndarray, word_bits: int = 64, with_bits: bool = True):
    """O3/O4: all (u, v), u < v, dist = 1, in (u, v) order.

    Returns (uv (E, 2) uint32, bit (E,) uint16, offsets (n+1,) int64)."""
    cells = np.ascontiguousarray(cells)
    nc, W = cells.shape
    offsets = np.zeros(nc + 1, dtype=np.int64)
    E = lib().cgo_edges(_p(cells), nc, word_bits, W, 0, None, None, _p(offsets), None)
    assert E >= 0
    uv = np.zeros((E, 2), dtype=np.uint32)
    bit = np.zeros(E, dtype=np.uint16)
    E2 = lib().cgo_edges(_p(cells), nc, word_bits, W, E, _p(uv),
                         _p(bit) if with_bits else None, None, None)
    assert E2 == E
    return uv, bit, offsets


def edges_search(cells: np.ndarray, ell: int, word_bits: int = 64):
    """O3/O4 by Algorithm 4's search (flip each 0 bit, look the result up
    among the sorted cells).  Cells must be sorted and distinct.  Same
    result as ``edges``; used where the all-pairs scan is too slow.

    Returns (uv (E, 2) uint32, bit (E,) uint16, offsets (n+1,) int64)."""
    cells = np.ascontiguousarray(cells)
    nc, W = cells.shape
    offsets = np.zeros(nc + 1, dtype=np.int64)
    E = lib().cgo_edges_search(_p(cells), nc, ell, word_bits, W, 0, None, None, _p(offsets), None)
    assert E >= 0
    uv = np.zeros((E, 2), dtype=np.uint32)
    bit = np.zeros(E, dtype=np.uint16)
    E2 = lib().cgo_edges_search(_p(cells), nc, ell, word_bits, W, E, _p(uv), _p(bit), None, None)
    assert E2 == E
    return uv, bit, offsets


def neighbors_of(cells: np.ndarray, sample: np.ndarray, word_bits: int = 64, max_deg: int = 4096):
    """All neighbors (both directions) of the sampled cells, by full scan."""
    cells = np.ascontiguousarray(cells)
    nc, W = cells.shape
    sample = np.ascontiguousarray(sample, dtype=np.int64)
    cnt = np.zeros(len(sample), dtype=np.uint32)
    ids = np.zeros((len(sample), max_deg), dtype=np.uint32)
    lib().cgo_neighbors_of(_p(cells), nc, word_bits, W, _p(sample), len(sample), max_deg,
                           _p(cnt), _p(ids))
    return [ids[s, :min(int(cnt[s]), max_deg)].copy() for s in range(len(sample))], cnt


def d1_queries(cells: np.ndarray, queries: np.ndarray, word_bits: int = 64):
    """O5: (count, self, mask) for arbitrary query rows."""
    cells = np.ascontiguousarray(cells)
    queries = np.ascontiguousarray(queries)
    nc, W = cells.shape
    nq = queries.shape[0]
    count = np.zeros(nq, dtype=np.uint32)
    self_ = np.zeros(nq, dtype=np.uint32)
    mask = np.zeros((nq, W), dtype=cells.dtype)
    lib().cgo_d1_queries(_p(cells), nc, _p(queries), nq, word_bits, W,
                         _p(count), _p(self_), _p(mask))
    return count, self_, mask


def ref_dists(cells: np.ndarray, refs: np.ndarray, word_bits: int = 64) -> np.ndarray:
    """Algorithm 1: D[d, j] = dist(refs[d], cells[j])."""
    cells = np.ascontiguousarray(cells)
    refs = np.ascontiguousarray(refs)
    nc, W = cells.shape
    h = refs.shape[0]
    D = np.zeros((h, nc), dtype=np.uint32)
    lib().cgo_ref_dists(_p(cells), nc, _p(refs), h, word_bits, W, _p(D))
    return D


def edges_heuristic(cells: np.ndarray, ref_ids, word_bits: int = 64):
    """Algorithm 2 with the corrected (*) filter, sequential."""
    cells = np.ascontiguousarray(cells)
    nc, W = cells.shape
    ref_ids = np.ascontiguousarray(np.asarray(ref_ids, dtype=np.int64))
    E = lib().cgo_edges_heuristic(_p(cells), nc, word_bits, W, _p(ref_ids), len(ref_ids),
                                  0, None, None)
    uv = np.zeros((E, 2), dtype=np.uint32)
    bit = np.zeros(E, dtype=np.uint16)
    lib().cgo_edges_heuristic(_p(cells), nc, word_bits, W, _p(ref_ids), len(ref_ids),
                              E, _p(uv), _p(bit))
    return uv, bit


def tree_levels(cells: np.ndarray, ell: int, r: int, word_bits: int = 64, nodes: bool = False):
    """Algorithm 3 on sorted distinct cells: level sizes (and optionally nodes)."""
    cells = np.ascontiguousarray(cells)
    nc, W = cells.shape
    depth = -(-ell // r)
    sizes = np.zeros(depth + 1, dtype=np.int64)
    total = lib().cgo_tree_levels(_p(cells), nc, ell, word_bits, W, r, _p(sizes), None, None, None)
    assert total >= 0
    if not nodes:
        return sizes
    nf = np.zeros(total, dtype=np.int64)
    nl = np.zeros(total, dtype=np.int64)
    nd = np.zeros(total, dtype=np.int32)
    lib().cgo_tree_levels(_p(cells), nc, ell, word_bits, W, r, _p(sizes), _p(nf), _p(nl), _p(nd))
    return sizes, nf, nl, nd


def digits(row: np.ndarray, ell: int, r: int, word_bits: int = 64) -> np.ndarray:
    row = np.ascontiguousarray(row)
    out = np.zeros(-(-ell // r), dtype=np.int32)
    lib().cgo_digits(_p(row), ell, word_bits, r, _p(out))
    return out


def dist(a: np.ndarray, b: np.ndarray, word_bits: int = 64) -> int:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return int(lib().cgo_dist(_p(a), _p(b), word_bits, a.shape[-1]))


def dist_bitwise(a: np.ndarray, b: np.ndarray, ell: int, word_bits: int = 64) -> int:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return int(lib().cgo_dist_bitwise(_p(a), _p(b), ell, word_bits))


def cell_graph(bits_or_rows: np.ndarray, ell: int, word_bits: int = 64, packed: bool = False):
    """Whole path on the CPU: (cells, row_to_cell, uv, bit, offsets)."""
    rows = bits_or_rows if packed else pack(bits_or_rows, word_bits)
    cells, r2c = dedup(rows, ell, word_bits)
    uv, bit, off = edges(cells, word_bits)
    return cells, r2c, uv, bit, off


def adjacency(n: int, uv: np.ndarray):
    """O6: undirected adjacency lists of the edge list: (adj_off (n+1,) int64,
    adj (2E,) uint32), each cell's neighbours ascending."""
    uv = np.ascontiguousarray(uv, dtype=np.uint32).reshape(-1, 2)
    E = uv.shape[0]
    adj_off = np.zeros(n + 1, dtype=np.int64)
    adj = np.zeros(max(2 * E, 1), dtype=np.uint32)
    assert lib().cgo_adjacency(n, E, _p(uv), _p(adj_off), _p(adj)) == 0
    return adj_off, adj[:2 * E]


def bfs(n: int, uv: np.ndarray, source: int):
    """O6: breadth-first search from `source`: (dist, parent, levels); dist and
    parent are 0xFFFFFFFF for unreached cells."""
    adj_off, adj = adjacency(n, uv)
    dist = np.zeros(n, dtype=np.uint32)
    parent = np.zeros(n, dtype=np.uint32)
    if adj.size == 0:
        adj = np.zeros(1, dtype=np.uint32)
    far = lib().cgo_bfs(n, _p(adj_off), _p(adj), source, _p(dist), _p(parent))
    assert far >= 0
    return dist, parent, int(far)


def philox4x64(counter, key) -> np.ndarray:
    """O7: one Philox4x64-10 block (4 x uint64) for a counter (4) and key (2)."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().cgo_philox4x64(_p(c), _p(k), _p(out))
    return out


def sample_point(i: int, seed: int, scene: int, lohi) -> np.ndarray:
    lohi = np.ascontiguousarray(lohi, dtype=np.float64)
    p = np.zeros(3, dtype=np.float64)
    lib().cgo_sample_point(i, seed, scene, _p(lohi), _p(p))
    return p


def sample_signs(planes: np.ndarray, n: int, seed: int, scene: int, lohi) -> np.ndarray:
    """O7: (n, ell) uint8 signs of n sampled points against planes (ell, 4)."""
    planes = np.ascontiguousarray(planes, dtype=np.float64).reshape(-1, 4)
    lohi = np.ascontiguousarray(lohi, dtype=np.float64)
    ell = planes.shape[0]
    bits = np.zeros((n, ell), dtype=np.uint8)
    assert lib().cgo_sample_signs(_p(planes), ell, n, seed, scene, _p(lohi), _p(bits)) == 0
    return bits
