"""Device-resident dictionary service (the abstract and Section 1 offer the
paper's search tree as a GPU dictionary for sets of long vectors over a
constant-size alphabet, useful on its own; Section 3.2: Algorithm 4 queries
it by flipping one position at a time).

A ``DictService`` keeps one set of cells and its dictionary in HBM and
answers batches of queries through ``cg_neighbors_d1``: for each query
vector, its own cell id (membership) and which one-position flips are
cells.  ``insert`` adds vectors by rebuilding (the current cells and the new
rows deduplicated together, then the dictionary rebuilt), so ids stay ranks
in lexicographic order.  ``QueryServer`` serves a trace of query requests
with continuous batching: every launch takes all requests that have arrived
(up to a batch limit), copies their vectors from pinned memory, queries, and
returns the results to the host.

Only buffer management and argument marshalling live here; every step of
the computation is a ``libcellgraph`` call.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as B


class DictService:
    def __init__(self, ell: int, word_bits: int = 64, capacity: int = 1 << 20,
                 params: B.DictParams | None = None, device: str = "cuda"):
        self.lay = B.make_layout(ell, word_bits)
        self.word_bits = word_bits
        self.cap = int(capacity)
        self.params = params if params is not None else B.cg_dict_params_default()
        self.device = torch.device(device)
        wdt = B.word_dtype(word_bits)
        W = self.lay.words
        self.rows = torch.empty((self.cap, W), dtype=wdt, device=self.device)   # dedup input
        self.cells = torch.empty((self.cap, W), dtype=wdt, device=self.device)
        self.r2c = torch.empty(self.cap, dtype=torch.int32, device=self.device)
        self.ncells = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.ws_bytes = B.cg_dedup_workspace(self.cap, self.lay)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.dict_bytes = B.cg_dict_size(self.cap, self.lay, self.params)
        self.dict_mem = torch.empty(self.dict_bytes, dtype=torch.uint8, device=self.device)
        self.dict = None
        self.n = 0  # cells, as last read back

    def _rebuild(self, m: int, stream=None) -> torch.Tensor:
        B.cg_dedup(self.rows, m, self.lay, self.cells, self.r2c, self.ncells, self.ws, self.ws_bytes, stream)
        self.dict = B.cg_dict_build(self.cells, self.ncells, self.cap, self.lay, self.params, self.dict_mem,
                                    self.dict_bytes, stream)
        torch.cuda.synchronize()
        self.n = int(self.ncells.item())
        return self.r2c[:m]

    def build(self, rows: torch.Tensor, stream=None) -> torch.Tensor:
        """Cells of `rows` (m x words, device) and the dictionary over them;
        returns each row's cell id (device, int32 view of uint32)."""
        m = rows.shape[0]
        if m > self.cap:
            raise ValueError(f"{m} rows exceed the capacity {self.cap}")
        self.rows[:m].copy_(rows)
        return self._rebuild(m, stream)

    def insert(self, rows: torch.Tensor, stream=None) -> torch.Tensor:
        """Insert by rebuild: the cells so far and `rows` are deduplicated
        together.  Returns the new ids of the inserted rows; ids of existing
        cells move to their new ranks."""
        m = rows.shape[0]
        if self.n + m > self.cap:
            raise ValueError(f"{self.n} cells + {m} rows exceed the capacity {self.cap}")
        n0 = self.n
        self.rows[:n0].copy_(self.cells[:n0])
        self.rows[n0:n0 + m].copy_(rows)
        ids = self._rebuild(n0 + m, stream)
        return ids[n0:n0 + m]

    def query(self, q: torch.Tensor, self_id=None, count=None, mask=None, stream=None):
        """Enqueue queries (no host wait): self_id (uint32 as int32; 0xFFFFFFFF
        for non-members), count of one-flip neighbours that are cells, and the
        flip mask (words per query)."""
        B.cg_neighbors_d1(self.dict, q, q.shape[0], count, self_id, mask, stream)


class QueryServer:
    """Continuous batching of query requests against a DictService.  A
    request is a block of query vectors; a launch takes every request that
    has arrived (up to ``max_batch`` vectors), so latency is the wait for
    the running launch plus one launch."""

    def __init__(self, svc: DictService, max_batch: int = 1 << 16):
        self.svc = svc
        self.max_batch = int(max_batch)
        W = svc.lay.words
        wdt = B.word_dtype(svc.word_bits)
        dev = svc.device
        self.h_q = torch.empty((self.max_batch, W), dtype=wdt).pin_memory()
        self.d_q = torch.empty((self.max_batch, W), dtype=wdt, device=dev)
        self.d_self = torch.empty(self.max_batch, dtype=torch.int32, device=dev)
        self.d_count = torch.empty(self.max_batch, dtype=torch.int32, device=dev)
        self.h_self = torch.empty(self.max_batch, dtype=torch.int32).pin_memory()
        self.h_count = torch.empty(self.max_batch, dtype=torch.int32).pin_memory()

    def serve(self, arrivals: np.ndarray, requests: list[np.ndarray]):
        """arrivals: seconds from start (ascending); requests[i]: (k_i, words)
        host array.  Returns (latencies s, results [(self, count)], wall s)."""
        n = len(arrivals)
        lat = np.zeros(n)
        res = [None] * n
        i = 0
        t0 = time.perf_counter()
        while i < n:
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(min(arrivals[i] - now, 1e-4))
                continue
            # every arrived request, up to the batch limit
            j, tot = i, 0
            while j < n and arrivals[j] <= now and tot + requests[j].shape[0] <= self.max_batch:
                tot += requests[j].shape[0]
                j += 1
            if j == i:  # a request larger than a whole batch is refused
                raise ValueError("request larger than max_batch")
            off = 0
            hq = self.h_q.numpy()
            for r in range(i, j):
                k = requests[r].shape[0]
                hq[off:off + k] = requests[r].view(hq.dtype)
                off += k
            self.d_q[:tot].copy_(self.h_q[:tot], non_blocking=True)
            self.svc.query(self.d_q[:tot], self.d_self, self.d_count)
            self.h_self[:tot].copy_(self.d_self[:tot], non_blocking=True)
            self.h_count[:tot].copy_(self.d_count[:tot], non_blocking=True)
            torch.cuda.synchronize()
            done = time.perf_counter() - t0
            hs, hc = self.h_self.numpy(), self.h_count.numpy()
            off = 0
            for r in range(i, j):
                k = requests[r].shape[0]
                res[r] = (hs[off:off + k].view(np.uint32).copy(), hc[off:off + k].view(np.uint32).copy())
                lat[r] = done - arrivals[r]
                off += k
            i = j
        return lat, res, time.perf_counter() - t0
