"""Pure numpy / Python restatement of the oracle, used only to pin the C oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

It reaches the same results by different routes, so that a mistake in one
(a dropped term, a wrong index, a reversed bit order) shows up as a mismatch:

* packing goes through ``numpy.packbits`` (big-endian bit order) and a byte
  swap into machine words, not a per-bit loop;
* sort + unique is ``numpy.unique(axis=0, return_inverse=True)`` on the 0/1
  byte matrix, whose row order is lexicographic with column 0 first
  (Section 3.2, the sorting step; Section 2.2 on multisets);
* edges are found on Python integers: with x(0) as the most significant bit,
  two cells are at distance 1 (Section 1.1, Section 2.2) iff their XOR is a
  power of two, and the differing position is l - bit_length(xor).
"""
from __future__ import annotations

import numpy as np


def pack_np(bits: np.ndarray, word_bits: int) -> np.ndarray:
    bits = (np.asarray(bits) != 0).astype(np.uint8)
    n, ell = bits.shape
    W = max(1, -(-ell // word_bits))
    padded = np.zeros((n, W * word_bits), dtype=np.uint8)
    padded[:, :ell] = bits
    by = np.packbits(padded, axis=1, bitorder="big")  # (n, W*word_bits/8), MSB first
    dt = ">u8" if word_bits == 64 else ">u4"
    words = by.view(dt).astype(np.uint64 if word_bits == 64 else np.uint32)
    return words.reshape(n, W)


def unique_np(bits: np.ndarray):
    bits = (np.asarray(bits) != 0).astype(np.uint8)
    if bits.shape[0] == 0:
        return bits.copy(), np.zeros(0, dtype=np.int64)
    cells, inv = np.unique(bits, axis=0, return_inverse=True)
    return cells, inv.reshape(-1)


def to_int(row_bits) -> int:
    v = 0
    for b in row_bits:
        v = (v << 1) | int(b != 0)
    return v


def edges_int(cells_bits: np.ndarray):
    """Edges of the cell graph by the power-of-two XOR test on integers."""
    ell = cells_bits.shape[1]
    vals = [to_int(r) for r in cells_bits]
    out = []
    for u in range(len(vals)):
        for v in range(u + 1, len(vals)):
            x = vals[u] ^ vals[v]
            if x and (x & (x - 1)) == 0:
                out.append((u, v, ell - x.bit_length()))
    return out


def cell_graph_np(bits: np.ndarray):
    cells, inv = unique_np(bits)
    return cells, inv, edges_int(cells)
