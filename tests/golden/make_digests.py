"""Writes the oracle's digests of the long-vector workload and of the 512
scenes of the batch workload (also the pool of the served trace).

Calls only ``oracle`` (the CPU reference) and ``inputs`` (the seeded
generators); nothing here comes from the HIP library.  For each workload the
oracle's cells, row_to_cell, edges (u, v), differing positions and CSR
offsets are reduced to SHA-256 digests of their raw little-endian bytes:
cells as packed rows (uint64 words for the long vectors, uint32 words,
ceil(l / 32) per row, for the plane scenes), row_to_cell uint32, uv uint32
(E, 2), bit uint16, offsets int64.

Edges of the plane scenes come from the all-pairs scan (the definition,
Section 2.2); those of the long vectors (4,194,304 cells, 8.8e12 pairs)
from the search form of Algorithm 4 (``oracle.edges_search``), which the
CPU pins check against the all-pairs scan.

  python tests/golden/make_digests.py long     # about a minute on 8 cores
  python tests/golden/make_digests.py batch    # the 512 scenes
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1503_06029_amd import inputs  # noqa: E402

LONG_FILE = os.path.join(HERE, "long_vectors_digest.txt")
BATCH_FILE = os.path.join(HERE, "batch_scenes_digest.txt")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def long_vectors():
    t0 = time.time()
    rows = inputs.long_vectors()
    cells, r2c = oracle.dedup(rows, 1024, 64)
    uv, bit, off = oracle.edges_search(cells, 1024, 64)
    lines = [
        "# oracle digests of the long-vector workload (inputs.long_vectors()):",
        "# 4,613,734 rows of 1024 bits as 16 uint64 words; written by make_digests.py",
        f"rows {rows.shape[0]}",
        f"cells {cells.shape[0]} {sha(cells.astype('<u8'))}",
        f"row_to_cell {sha(r2c.astype('<u4'))}",
        f"edges {uv.shape[0]}",
        f"uv {sha(uv.astype('<u4'))}",
        f"bit {sha(bit.astype('<u2'))}",
        f"offsets {sha(off.astype('<i8'))}",
    ]
    with open(LONG_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"long vectors: {cells.shape[0]} cells, {uv.shape[0]} edges, {time.time() - t0:.1f} s")


def scene_record(i: int) -> str:
    R = inputs.batch_scene(i)
    n, ell = R.shape
    rows = oracle.pack(R, 32)
    cells, r2c = oracle.dedup(rows, ell, 32)
    uv, bit, off = oracle.edges(cells, 32)
    return (f"{i} {ell} {n} {cells.shape[0]} {uv.shape[0]} {sha(cells.astype('<u4'))} "
            f"{sha(r2c.astype('<u4'))} {sha(uv.astype('<u4'))} {sha(bit.astype('<u2'))} {sha(off.astype('<i8'))}")


def batch(first: int = 0, last: int = inputs.BATCH_SCENES):
    t0 = time.time()
    recs = []
    for i in range(first, last):
        recs.append(scene_record(i))
        print(recs[-1][:60], f"{time.time() - t0:.0f} s", flush=True)
    head = ["# oracle digests of the 512 scenes of the batch workload (inputs.batch_scene(i)),",
            "# packed as ceil(l / 32) uint32 words; written by make_digests.py",
            "# scene l n cells edges sha(cells) sha(row_to_cell) sha(uv) sha(bit) sha(offsets)"]
    with open(BATCH_FILE, "w") as f:
        f.write("\n".join(head + recs) + "\n")


def read_long():
    out = {}
    with open(LONG_FILE) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = v
    return out


def read_batch():
    out = {}
    with open(BATCH_FILE) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            out[int(p[0])] = {"ell": int(p[1]), "n": int(p[2]), "ncells": int(p[3]), "nedges": int(p[4]),
                              "cells": p[5], "row_to_cell": p[6], "uv": p[7], "bit": p[8], "offsets": p[9]}
    return out


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "long"
    if what == "long":
        long_vectors()
    elif what == "batch":
        batch()
    else:
        raise SystemExit("usage: make_digests.py long|batch")
