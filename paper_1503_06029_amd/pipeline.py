"""Whole-path driver over the C ABI: allocates torch device buffers once and
runs pack -> dedup -> dictionary -> edges on the current stream.

Only buffer management and argument marshalling live here; every step of
the computation is a ``libcellgraph`` call (see ``binding.py``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _np_words(t: torch.Tensor, word_bits: int) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint64 if word_bits == 64 else np.uint32)


class CellGraph:
    """Buffers and calls for one scene shape (n_rows x ell, word_bits).

    ``run(packed)`` enqueues dedup, dictionary build and edge emission;
    ``run_bits(bits)`` packs a uint8 sign matrix first.  Results stay on the
    device until ``fetch()``."""

    def __init__(self, n_rows: int, ell: int, word_bits: int = 64, params: B.DictParams | None = None,
                 edge_cap: int | None = None, with_bits: bool = True, with_row_to_cell: bool = True,
                 with_offsets: bool = True, device: str = "cuda"):
        self.n = int(n_rows)
        self.lay = B.make_layout(ell, word_bits)
        self.word_bits = word_bits
        self.params = params if params is not None else B.cg_dict_params_default()
        self.device = torch.device(device)
        wdt = B.word_dtype(word_bits)
        W = self.lay.words
        m = max(self.n, 1)
        dev = self.device
        self.packed = torch.empty((m, W), dtype=wdt, device=dev)
        self.cells = torch.empty((m, W), dtype=wdt, device=dev)
        self.r2c = torch.empty(m, dtype=torch.int32, device=dev) if with_row_to_cell else None
        self.ncells = torch.zeros(1, dtype=torch.int64, device=dev)
        # the fused dedup + dictionary build needs a little more than dedup alone
        self.ws_dedup_bytes = max(B.cg_dedup_workspace(self.n, self.lay), B.cg_dedup_dict_workspace(self.n, self.lay))
        self.ws_dedup = torch.empty(self.ws_dedup_bytes, dtype=torch.uint8, device=dev)
        self.dict_bytes = B.cg_dict_size(self.n, self.lay, self.params)
        self.dict_mem = torch.empty(self.dict_bytes, dtype=torch.uint8, device=dev)
        if edge_cap is None:
            edge_cap = max(1024, 2 * self.n)
        self.edge_cap = int(edge_cap)
        self.with_bits = with_bits
        self.uv = torch.empty((max(self.edge_cap, 1), 2), dtype=torch.int32, device=dev)
        self.bit = torch.empty(max(self.edge_cap, 1), dtype=torch.int16, device=dev) if with_bits else None
        self.offsets = torch.empty(m + 1, dtype=torch.int64, device=dev) if with_offsets else None
        self.nedges = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.dict = None
        self.ws_edges = None
        self.ws_edges_bytes = 0

    # ------------------------------------------------------------- steps
    def pack(self, bits: torch.Tensor, stream=None):
        assert bits.dtype == torch.uint8 and bits.shape[0] == self.n and bits.shape[1] == self.lay.ell
        B.cg_pack(bits, self.n, bits.stride(0), self.lay, self.packed, stream)

    def sample(self, planes: torch.Tensor, seed: int, scene: int, box, stream=None):
        """Fill the packed rows with n sampled points' sign vectors
        (planes: (ell, 4) float64 on the device; box: lo0, lo1, lo2, hi0, hi1, hi2)."""
        B.cg_sample_pack(planes, self.n, seed, scene, box, self.lay, self.packed, stream)

    def dedup(self, packed: torch.Tensor | None = None, stream=None):
        src = self.packed if packed is None else packed
        B.cg_dedup(src, self.n, self.lay, self.cells, self.r2c, self.ncells, self.ws_dedup,
                   self.ws_dedup_bytes, stream)

    def dedup_dict(self, packed: torch.Tensor | None = None, stream=None):
        """dedup() and build_dict() as one fused call (same results)."""
        src = self.packed if packed is None else packed
        self.dict = B.cg_dedup_dict(src, self.n, self.lay, self.cells, self.r2c, self.ncells, self.ws_dedup,
                                    self.ws_dedup_bytes, self.params, self.dict_mem, self.dict_bytes, stream)
        self._edges_ws()

    def build_dict(self, stream=None):
        self.dict = B.cg_dict_build(self.cells, self.ncells, self.n, self.lay, self.params, self.dict_mem,
                                    self.dict_bytes, stream)
        self._edges_ws()

    def _edges_ws(self):
        need = B.cg_edges_workspace(self.dict, self.edge_cap)
        if self.ws_edges is None or need > self.ws_edges_bytes:
            self.ws_edges = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_edges_bytes = need

    def edges(self, stream=None):
        B.cg_edges(self.dict, self.uv, self.bit, self.edge_cap, self.nedges, self.offsets, self.ws_edges,
                   self.ws_edges_bytes, self.status, stream)

    def run(self, packed: torch.Tensor | None = None, stream=None):
        self.dedup(packed, stream)
        self.build_dict(stream)
        self.edges(stream)

    def run_bits(self, bits: torch.Tensor, stream=None):
        self.pack(bits, stream)
        self.run(None, stream)

    def grow_edges(self, cap: int):
        self.edge_cap = int(cap)
        self.uv = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
        if self.with_bits:
            self.bit = torch.empty(max(cap, 1), dtype=torch.int16, device=self.device)
        need = B.cg_edges_workspace(self.dict, self.edge_cap)
        if need > self.ws_edges_bytes:
            self.ws_edges = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_edges_bytes = need

    def run_checked(self, packed=None, stream=None):
        """run(), then re-run cg_edges with a larger capacity if it overflowed."""
        self.run(packed, stream)
        torch.cuda.synchronize()
        if int(self.status.item()) == B.CG_ECAPACITY:
            self.grow_edges(int(self.nedges.item()))
            self.edges(stream)
            torch.cuda.synchronize()
        assert int(self.status.item()) == B.CG_OK

    # ------------------------------------------------------------ results
    def fetch(self):
        torch.cuda.synchronize()
        nc = int(self.ncells.item())
        E = int(self.nedges.item())
        out = {
            "ncells": nc,
            "nedges": E,
            "status": int(self.status.item()),
            "cells": _np_words(self.cells[:nc], self.word_bits),
            "uv": self.uv[:min(E, self.edge_cap)].cpu().numpy().view(np.uint32),
        }
        if self.r2c is not None:
            out["row_to_cell"] = self.r2c[:self.n].cpu().numpy().view(np.uint32)
        if self.bit is not None:
            out["bit"] = self.bit[:min(E, self.edge_cap)].cpu().numpy().view(np.uint16)
        if self.offsets is not None:
            out["offsets"] = self.offsets[:nc + 1].cpu().numpy()
        return out

    def neighbors_d1(self, queries: torch.Tensor, stream=None):
        nq = queries.shape[0]
        dev = self.device
        cnt = torch.empty(max(nq, 1), dtype=torch.int32, device=dev)
        me = torch.empty(max(nq, 1), dtype=torch.int32, device=dev)
        mask = torch.empty((max(nq, 1), self.lay.words), dtype=B.word_dtype(self.word_bits), device=dev)
        B.cg_neighbors_d1(self.dict, queries, nq, cnt, me, mask, stream)
        torch.cuda.synchronize()
        return (cnt[:nq].cpu().numpy().view(np.uint32), me[:nq].cpu().numpy().view(np.uint32),
                _np_words(mask[:nq], self.word_bits))


class GraphSearch:
    """Undirected adjacency (CSR) of a built CellGraph's edges and
    breadth-first search over it, all in device buffers.  The CellGraph must
    have been run with offsets and must outlive this object."""

    UNREACHED = 0xFFFFFFFF

    def __init__(self, g: CellGraph):
        if g.offsets is None:
            raise ValueError("GraphSearch needs a CellGraph made with offsets")
        self.g = g
        dev = g.device
        self.ncap = g.n
        self.ecap = g.edge_cap
        self.adj_off = torch.empty(self.ncap + 1, dtype=torch.int64, device=dev)
        self.adj = torch.empty(max(2 * self.ecap, 1), dtype=torch.int32, device=dev)
        self.csr_status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_csr_bytes = B.cg_graph_csr_workspace(self.ncap, self.ecap)
        self.ws_csr = torch.empty(self.ws_csr_bytes, dtype=torch.uint8, device=dev)
        self.dist = torch.empty(max(self.ncap, 1), dtype=torch.int32, device=dev)
        self.parent = torch.empty(max(self.ncap, 1), dtype=torch.int32, device=dev)
        self.levels = torch.zeros(1, dtype=torch.int32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_bfs_bytes = B.cg_bfs_workspace(self.ncap)
        self.ws_bfs = torch.empty(self.ws_bfs_bytes, dtype=torch.uint8, device=dev)

    def build(self, stream=None):
        g = self.g
        B.cg_graph_csr(g.uv, g.offsets, g.ncells, self.ncap, g.nedges, self.ecap, self.adj_off, self.adj,
                       self.csr_status, self.ws_csr, self.ws_csr_bytes, stream)

    def bfs(self, source: int, max_levels: int = 64, resume: bool = False, stream=None):
        """Enqueue max_levels levels of the search (no host wait)."""
        B.cg_bfs(self.adj_off, self.adj, self.g.ncells, self.ncap, source, max_levels, resume, self.dist,
                 self.parent, self.levels, self.status, self.ws_bfs, self.ws_bfs_bytes, stream)

    def bfs_complete(self, source: int, chunk: int = 64, stream=None) -> int:
        """Search until the frontier is empty, checking the status after each
        chunk of levels; returns the final status."""
        self.bfs(source, chunk, False, stream)
        while True:
            torch.cuda.synchronize()
            st = int(self.status.item())
            if st != B.CG_ECAPACITY:
                return st
            self.bfs(source, chunk, True, stream)

    def capture(self, source: int, max_levels: int):
        """Record build() and a max_levels-level search from `source` into
        one graph; replay() reruns both without per-launch host work."""
        self.graph = torch.cuda.CUDAGraph()
        cap_stream = torch.cuda.Stream()
        cap_stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=cap_stream):
            self.build()
            self.bfs(source, max_levels, False)
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()

    def path(self, target: int, stream=None) -> np.ndarray:
        """Cells of the shortest path source .. target along the parents."""
        cap = max(int(self.levels.item()) + 1, 1)
        out = torch.empty(cap, dtype=torch.int32, device=self.g.device)
        ln = torch.zeros(1, dtype=torch.int64, device=self.g.device)
        B.cg_bfs_path(self.dist, self.parent, self.g.ncells, self.ncap, target, out, cap, ln, stream)
        torch.cuda.synchronize()
        L = int(ln.item())
        return out[:min(L, cap)].cpu().numpy().view(np.uint32).copy() if L <= cap else None

    def fetch(self):
        torch.cuda.synchronize()
        nc = int(self.g.ncells.item())
        off = self.adj_off[:nc + 1].cpu().numpy()
        return {
            "csr_status": int(self.csr_status.item()),
            "adj_off": off,
            "adj": self.adj[:int(off[-1]) if nc else 0].cpu().numpy().view(np.uint32),
            "dist": self.dist[:nc].cpu().numpy().view(np.uint32),
            "parent": self.parent[:nc].cpu().numpy().view(np.uint32),
            "levels": int(self.levels.item()),
            "status": int(self.status.item()),
        }


def to_device_words(rows: np.ndarray, device="cuda") -> torch.Tensor:
    """Host packed rows (uint32 / uint64) -> device tensor of the same bytes."""
    rows = np.ascontiguousarray(rows)
    if rows.dtype == np.uint64:
        t = torch.from_numpy(rows.view(np.int64))
    elif rows.dtype == np.uint32:
        t = torch.from_numpy(rows.view(np.int32))
    else:
        raise TypeError(rows.dtype)
    return t.to(device)


def cell_graph(data: np.ndarray, ell: int, word_bits: int = 64, packed: bool = False,
               params: B.DictParams | None = None, device="cuda"):
    """One scene end to end on the GPU; returns the fetched host results."""
    n = data.shape[0]
    g = CellGraph(n, ell, word_bits, params, device=device)
    if packed:
        g.run_checked(to_device_words(data, device))
    else:
        bits = torch.from_numpy(np.ascontiguousarray(data, dtype=np.uint8)).to(device)
        if n:
            g.pack(bits)
        g.run_checked()
    res = g.fetch()
    res["graph"] = g
    return res
