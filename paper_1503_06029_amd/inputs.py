"""Seeded synthetic inputs for the cell-graph path.

This module is shared by the tests, the oracle checks and the benchmark.  It
holds none of the method's arithmetic (no packing, sorting, deduplication or
distance work): it only draws scenes and sample points and evaluates which
side of each constraint a point lies on, the way a sample generator does
(Section 2.1, sample generators; Section 2.2, X may be a multiset).

The paper's own workloads (a sample generator over SO(3) rotations and
real-life scenes) are not available, so these stand in for them at the scale
the paper assumes (n up to a few million, l up to a few hundred):

* ``line_arrangement``: 32 random lines in the unit square, 10,000 uniform points;
* ``plane_arrangement``: 128 random planes in [-1, 1]^3, 1,000,000 uniform points;
* ``long_vectors``: 262,144 random 1024-bit base vectors, each with 15 neighbours made
  by flipping 15 distinct uniformly chosen bits, rows shuffled, 10% duplicate
  rows appended and shuffled again (4,613,734 rows, already packed as
  16 x uint64, most significant bit first);
* ``batch_scene``: one scene of the batched distribution (l uniform in 16..512
  random planes in R^3, sample count log-uniform in [1,000, 200,000]);
* ``served_trace``: Poisson arrivals at 2,000 scenes/s for 60 s over a pool of
  512 scenes of the batched distribution.

A sign is 1 iff the point satisfies the constraint a . p - c >= 0, computed
in float64 on the host.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 150306029


def _rng(workload: int, *extra: int) -> np.random.Generator:
    """Independent seeded stream per workload (0 lines, 1 plane arrangement,
    2 long vectors, 3 scene batch, 4 served trace) and sub-stream."""
    ss = np.random.SeedSequence(MASTER_SEED).spawn(5)[workload]
    for e in extra:
        ss = ss.spawn(e + 1)[e]
    return np.random.Generator(np.random.PCG64(ss))


def _signs(points: np.ndarray, normals: np.ndarray, offsets: np.ndarray,
           chunk: int = 1 << 16) -> np.ndarray:
    n = points.shape[0]
    ell = normals.shape[0]
    out = np.empty((n, ell), dtype=np.uint8)
    for s in range(0, n, chunk):
        r = points[s:s + chunk] @ normals.T - offsets[None, :]
        out[s:s + chunk] = r >= 0.0
    return out


def lines_in_square(rng: np.random.Generator, ell: int, n: int) -> np.ndarray:
    """l lines with normals uniform on the circle and offsets spread over the
    range that meets the unit square; n uniform points in [0, 1]^2."""
    theta = rng.uniform(0.0, 2.0 * np.pi, ell)
    a = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    corners = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    proj = a @ corners.T
    c = rng.uniform(proj.min(axis=1), proj.max(axis=1))
    pts = rng.uniform(0.0, 1.0, (n, 2))
    return _signs(pts, a, c)


def planes_in_cube(rng: np.random.Generator, ell: int, n: int) -> np.ndarray:
    """l planes with normals uniform on the sphere and offsets uniform in
    [-0.5, 0.5]; n uniform points in [-1, 1]^3."""
    g = rng.standard_normal((ell, 3))
    a = g / np.linalg.norm(g, axis=1, keepdims=True)
    c = rng.uniform(-0.5, 0.5, ell)
    pts = rng.uniform(-1.0, 1.0, (n, 3))
    return _signs(pts, a, c)


def line_arrangement() -> np.ndarray:
    """Lines workload: uint8 (10000, 32) sign matrix of 10,000 points in the unit
    square against 32 lines, duplicates kept."""
    return lines_in_square(_rng(0), 32, 10_000)


def plane_arrangement(n: int = 1_000_000) -> np.ndarray:
    """Plane-arrangement workload: uint8 (1e6, 128) sign matrix of 10^6 points
    in [-1, 1]^3 against 128 planes."""
    return planes_in_cube(_rng(1), 128, n)


def flip_bit_u64(rows: np.ndarray, bit: np.ndarray) -> None:
    """In place: flip vector position ``bit[i]`` of packed uint64 row
    ``rows[i]`` (word bit // 64, bit 63 - bit % 64: most significant first)."""
    w = bit // 64
    m = np.left_shift(np.uint64(1), (63 - (bit % 64)).astype(np.uint64))
    idx = np.arange(rows.shape[0])
    rows[idx, w] ^= m


def long_vectors(n_bases: int = 262_144, ell: int = 1024, n_flips: int = 15,
       dup_frac: float = 0.10, seed_extra: int = 0) -> np.ndarray:
    """Long-vector workload: packed uint64 rows (n_bases * 16 * 1.1, ell / 64).

    Bases are uniform in [2]^l; each gets ``n_flips`` neighbours made by
    flipping distinct uniformly chosen positions.  Rows are shuffled, then
    round(dup_frac * rows) duplicates drawn uniformly with replacement are
    appended and everything is shuffled again."""
    assert ell % 64 == 0
    rng = _rng(2, seed_extra) if seed_extra else _rng(2)
    W = ell // 64
    base = rng.integers(0, np.iinfo(np.uint64).max, size=(n_bases, W),
                        dtype=np.uint64, endpoint=True)
    fam = n_flips + 1
    rows = np.repeat(base, fam, axis=0)  # row b*fam + 0 is the base itself
    chunk = 8192
    for s in range(0, n_bases, chunk):
        e = min(n_bases, s + chunk)
        keys = rng.random((e - s, ell), dtype=np.float32)
        picks = np.argpartition(keys, n_flips, axis=1)[:, :n_flips]  # distinct positions
        picks.sort(axis=1)
        for f in range(n_flips):
            sub = rows[s * fam + 1 + f:e * fam:fam]  # a view: flipped in place
            flip_bit_u64(sub, picks[:, f].astype(np.int64))
    rows = rows[rng.permutation(rows.shape[0])]
    n_dup = int(round(dup_frac * rows.shape[0]))
    dup = rows[rng.integers(0, rows.shape[0], n_dup)]
    rows = np.concatenate([rows, dup], axis=0)
    rows = rows[rng.permutation(rows.shape[0])]
    return np.ascontiguousarray(rows)


def long_vectors_expected(n_bases: int = 262_144, n_flips: int = 15):
    """Cells and edges of the long-vector workload by construction: bases and planted
    neighbours are all distinct, and the only distance-1 pairs are
    (base, planted neighbour), unless two independent uniform 1024-bit bases
    fall within distance 2 of each other (probability below 2^-900)."""
    return n_bases * (n_flips + 1), n_bases * n_flips


BATCH_SCENES = 512


def batch_scene_params(i: int):
    rng = _rng(3, i)
    ell = int(rng.integers(16, 512, endpoint=True))
    n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    return ell, n


def batch_scene(i: int) -> np.ndarray:
    """Scene i of the 512-scene batch workload: uint8 (n_i, l_i) sign matrix."""
    rng = _rng(3, i)
    ell = int(rng.integers(16, 512, endpoint=True))
    n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    return planes_in_cube(rng, ell, n)


def batch_scene_desc(i: int):
    """Scene i of the 512-scene batch workload as a description for the GPU sampler: the same l,
    n and planes as batch_scene(i) (rows (a0, a1, a2, c), float64), points to
    be drawn in [-1, 1]^3 with Philox key (MASTER_SEED, i).  Returns
    (planes, n, key)."""
    rng = _rng(3, i)
    ell = int(rng.integers(16, 512, endpoint=True))
    n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    g = rng.standard_normal((ell, 3))
    a = g / np.linalg.norm(g, axis=1, keepdims=True)
    c = rng.uniform(-0.5, 0.5, ell)
    return np.concatenate([a, c[:, None]], axis=1), n, (MASTER_SEED, i)


SAMPLE_BOX = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)


def served_trace(rate: float = 2000.0, seconds: float = 60.0, pool: int = BATCH_SCENES):
    """Served trace: (arrival times in s, scene index in the 512-scene pool)."""
    rng = _rng(4)
    gaps = rng.exponential(1.0 / rate, int(rate * seconds * 1.2) + 100)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    scene = rng.integers(0, pool, t.shape[0])
    return t, scene


def random_multiset(rng: np.random.Generator, n: int, ell: int, n_distinct: int | None = None,
                    p_one: float = 0.5) -> np.ndarray:
    """Small random multisets for tests: n rows drawn with replacement from
    n_distinct random vectors (or independent rows when n_distinct is None)."""
    if n_distinct is None:
        return (rng.random((n, ell)) < p_one).astype(np.uint8)
    pool = (rng.random((n_distinct, ell)) < p_one).astype(np.uint8)
    return pool[rng.integers(0, n_distinct, n)]


def clustered_multiset(rng: np.random.Generator, n_bases: int, ell: int, fam: int,
                       dups: int) -> np.ndarray:
    """Bases plus one-bit neighbours plus duplicates, as uint8 rows: many
    distance-1 pairs at every bit position, for tests of small shapes."""
    base = (rng.random((n_bases, ell)) < 0.5).astype(np.uint8)
    rows = [base]
    for _ in range(fam):
        nb = base.copy()
        k = rng.integers(0, ell, n_bases)
        nb[np.arange(n_bases), k] ^= 1
        rows.append(nb)
    rows = np.concatenate(rows, axis=0)
    if dups:
        rows = np.concatenate([rows, rows[rng.integers(0, rows.shape[0], dups)]], axis=0)
    return rows[rng.permutation(rows.shape[0])]
