"""Batched scenes: many independent scenes through one set of launches.

Scenes are grouped by width into classes (virtual rows of 2, 4, 8, 16 or 32
32-bit words: one tag word holding the scene number twice, then the
scene's vector).  Each class is one virtual scene for the ordinary
``cg_dedup`` / ``cg_dict_build`` / ``cg_edges`` calls; ``cg_batch_split``
finds every scene's slice and makes ids and positions scene-local.  Classes
run on their own streams and the whole batch can be captured into one HIP
graph (``BatchRunner.capture``), so a replay is a single graph launch.

Only buffer management and argument marshalling live here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B

CLASS_WORDS = (2, 4, 8, 16, 32)  # tag word + data words, a power of two
TAG_BITS = 32
MAX_ELL = 32 * (CLASS_WORDS[-1] - 1)  # longest vector a class holds

# Data bits of the default split per class: the P pass (flips at or after
# the split) sees groups of cells that agree on the tag and the first
# SPLIT_DATA planes, the S pass runs of cells that agree on the rest.  For
# arrangements of planes both stay small when each side holds a good share
# of a scene's planes; a class holds scenes of l in (32 (w/2 - 1), 32 (w - 1)].
SPLIT_DATA = {2: 16, 4: 32, 8: 64, 16: 128, 32: 256}


def default_params(words: int) -> B.DictParams:
    return B.cg_dict_params_default(split_bit=TAG_BITS + SPLIT_DATA[words])


def class_words(ell: int) -> int:
    need = 1 + -(-ell // 32)
    for w in CLASS_WORDS:
        if need <= w:
            return w
    raise ValueError(f"l = {ell} is too long for a batch class (max {32 * (CLASS_WORDS[-1] - 1)})")


def class_footprint(rows: int, scenes: int, nbytes: int, words: int, edge_cap: int | None = None) -> int:
    """Device bytes of one SceneBatch of `words`-word rows with capacity for
    `rows` rows, `scenes` scenes and `nbytes` sign bytes (the edge capacity
    defaults to SceneBatch's, 4 per row): buffers plus the dedup, dictionary
    and edge workspaces the library reports for those sizes."""
    lay = B.cg_batch_layout(32 * (words - 1))
    m = max(rows, 1)
    ecap = int(edge_cap if edge_cap is not None else max(4096, 4 * rows))
    params = default_params(words)
    tot = 0
    tot += 8 * (scenes + 1) + 8 * scenes * 3 + 4 * scenes + 16 * scenes  # scene tables
    tot += max(nbytes, 16)                                            # sign bytes
    tot += 2 * 4 * m * words + 4 * m                                  # packed rows, cells, row_to_cell
    tot += max(B.cg_dedup_workspace(rows, lay), B.cg_dedup_dict_workspace(rows, lay)) + B.cg_dict_size(rows, lay, params)
    tot += ecap * (8 + 2) + 8 * (m + 1)                               # uv, bit, offsets
    tot += B.cg_edges_workspace_for(rows, lay, params, ecap)
    tot += 16 * (scenes + 1)                                          # cell and edge offsets
    return int(tot)


class SceneBatch:
    """One width class: scenes of lengths ``ells`` and row counts ``ns``.

    Buffers are sized for capacities (rows, scenes, sign bytes, edges), so the
    same object can take another set of scenes with ``set_scenes`` (the
    serving loop reuses it batch after batch)."""

    def __init__(self, ells, ns, words: int, params: B.DictParams | None = None, edge_cap: int | None = None,
                 device="cuda", max_rows: int | None = None, max_scenes: int | None = None,
                 max_bytes: int | None = None):
        ells = np.asarray(ells, dtype=np.int32)
        ns = np.asarray(ns, dtype=np.int64)
        self.words = words
        self.lay = B.cg_batch_layout(32 * (words - 1))
        assert self.lay.words == words
        self.device = torch.device(device)
        dev = self.device
        self.cap_rows = int(max_rows if max_rows is not None else ns.sum())
        self.cap_scenes = int(max_scenes if max_scenes is not None else len(ells))
        self.cap_bytes = int(max_bytes if max_bytes is not None else (ns * ells).sum())
        m = max(self.cap_rows, 1)
        self.scene_rows = torch.zeros(self.cap_scenes + 1, dtype=torch.int64, device=dev)
        self.bits_off = torch.zeros(max(self.cap_scenes, 1), dtype=torch.int64, device=dev)
        self.scene_ell = torch.zeros(max(self.cap_scenes, 1), dtype=torch.int32, device=dev)
        # sampled scenes: each scene's first plane in a device plane pool and its generator key
        self.planes_off = torch.zeros(max(self.cap_scenes, 1), dtype=torch.int64, device=dev)
        self.keys = torch.zeros((max(self.cap_scenes, 1), 2), dtype=torch.int64, device=dev)
        self.bits = torch.empty(max(self.cap_bytes, 16), dtype=torch.uint8, device=dev)
        self.packed = torch.empty((m, words), dtype=torch.int32, device=dev)
        self.cells = torch.empty((m, words), dtype=torch.int32, device=dev)
        self.r2c = torch.empty(m, dtype=torch.int32, device=dev)
        self.ncells = torch.zeros(1, dtype=torch.int64, device=dev)
        # the fused build (taken with a chosen key width) needs a little more
        self.ws_dedup_bytes = max(B.cg_dedup_workspace(self.cap_rows, self.lay),
                                  B.cg_dedup_dict_workspace(self.cap_rows, self.lay))
        self.ws_dedup = torch.empty(self.ws_dedup_bytes, dtype=torch.uint8, device=dev)
        self.params = params if params is not None else default_params(words)
        self.dict_bytes = B.cg_dict_size(self.cap_rows, self.lay, self.params)
        self.dict_mem = torch.empty(self.dict_bytes, dtype=torch.uint8, device=dev)
        self.edge_cap = int(edge_cap if edge_cap is not None else max(4096, 4 * self.cap_rows))
        self.uv = torch.empty((self.edge_cap, 2), dtype=torch.int32, device=dev)
        self.bit = torch.empty(self.edge_cap, dtype=torch.int16, device=dev)
        self.offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)
        self.nedges = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cell_off = torch.zeros(self.cap_scenes + 1, dtype=torch.int64, device=dev)
        self.edge_off = torch.zeros(self.cap_scenes + 1, dtype=torch.int64, device=dev)
        self.dict = None
        self.ws_edges = None
        self.ws_edges_bytes = 0
        self.set_scenes(ells, ns)

    def set_sampled(self, ells, ns, planes_off, keys):
        """Point the batch at scenes described by planes (offsets into a
        device plane pool) and generator keys, to be sampled on the GPU."""
        self.set_scenes(ells, ns, check_bytes=False)
        k = self.n_scenes
        self.planes_off[:k].copy_(torch.from_numpy(np.asarray(planes_off, dtype=np.int64)))
        kk = np.asarray(keys, dtype=np.uint64).reshape(k, 2).view(np.int64)
        self.keys[:k].copy_(torch.from_numpy(np.ascontiguousarray(kk)))

    def set_scenes(self, ells, ns, check_bytes: bool = True):
        """Point the batch at a new set of scenes (within capacity)."""
        self.ells = np.asarray(ells, dtype=np.int32)
        self.ns = np.asarray(ns, dtype=np.int64)
        self.n_scenes = len(self.ells)
        assert 1 <= self.n_scenes <= self.cap_scenes
        rows = np.zeros(self.n_scenes + 1, dtype=np.int64)
        rows[1:] = np.cumsum(self.ns)
        bytes_per = self.ns * self.ells
        boff = np.zeros(self.n_scenes, dtype=np.int64)
        boff[1:] = np.cumsum(bytes_per)[:-1]
        self.n_rows = int(rows[-1])
        self.total_bytes = int(bytes_per.sum())
        assert self.n_rows <= self.cap_rows and (self.total_bytes <= self.cap_bytes or not check_bytes)
        assert int(self.ells.max()) <= 32 * (self.words - 1)
        self.scene_rows_h = rows
        self.bits_off_h = boff
        self.scene_rows[:self.n_scenes + 1].copy_(torch.from_numpy(rows))
        self.bits_off[:self.n_scenes].copy_(torch.from_numpy(boff))
        self.scene_ell[:self.n_scenes].copy_(torch.from_numpy(self.ells))

    def upload(self, scenes, stream=None):
        """Copy the scenes' uint8 sign matrices into the batch's byte buffer."""
        host = np.empty(self.total_bytes, dtype=np.uint8)
        for j, R in enumerate(scenes):
            assert R.shape == (self.ns[j], self.ells[j])
            o = self.bits_off_h[j]
            host[o:o + R.size] = np.ascontiguousarray(R, dtype=np.uint8).reshape(-1)
        if self.total_bytes:
            self.bits[:self.total_bytes].copy_(torch.from_numpy(host), non_blocking=False)

    def _edges_ws(self):
        need = B.cg_edges_workspace(self.dict, self.edge_cap)
        if self.ws_edges is None or need > self.ws_edges_bytes:
            self.ws_edges = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_edges_bytes = need

    def run(self, stream=None):
        B.cg_batch_pack(self.bits, self.bits_off, self.scene_ell, self.scene_rows, self.n_scenes, self.n_rows,
                        self.lay, self.packed, stream)
        self._last = ("bits",)
        self._run_path(stream)

    def rerun(self, stream=None):
        """Run the last batch again (its inputs are still in place), e.g.
        after grow_edges."""
        if self._last[0] == "bits":
            self.run(stream)
        else:
            self.run_sampled(self._last[1], self._last[2], stream)

    def run_sampled(self, planes, box, stream=None):
        """Sample the scenes set by set_sampled (plane pool `planes`, (P, 4)
        float64 on the device) straight into the packed rows, then the path."""
        B.cg_batch_sample_pack(planes, self.planes_off, self.scene_ell, self.scene_rows, self.keys, self.n_scenes,
                               self.n_rows, box, self.lay, self.packed, stream)
        self._last = ("sampled", planes, box)
        self._run_path(stream)

    def _run_path(self, stream=None):
        if self.params.key_bits:
            # a chosen sort-key width: the fused dedup + dictionary build
            self.dict = B.cg_dedup_dict(self.packed, self.n_rows, self.lay, self.cells, self.r2c, self.ncells,
                                        self.ws_dedup, self.ws_dedup_bytes, self.params, self.dict_mem,
                                        self.dict_bytes, stream)
        else:
            B.cg_dedup(self.packed, self.n_rows, self.lay, self.cells, self.r2c, self.ncells, self.ws_dedup,
                       self.ws_dedup_bytes, stream)
            self.dict = B.cg_dict_build(self.cells, self.ncells, self.n_rows, self.lay, self.params, self.dict_mem,
                                        self.dict_bytes, stream)
        self._edges_ws()  # allocates only when a larger batch needs more
        B.cg_edges(self.dict, self.uv, self.bit, self.edge_cap, self.nedges, self.offsets, self.ws_edges,
                   self.ws_edges_bytes, self.status, stream)
        B.cg_batch_split(self.dict, self.n_scenes, self.offsets, self.nedges, self.edge_cap, self.cell_off,
                         self.edge_off, True, self.uv, self.bit, self.r2c, self.scene_rows, self.n_rows, stream)

    def needed_edges(self) -> int:
        """Edge count of the last run (exact even when it overflowed)."""
        return int(self.nedges.item())

    def grow_edges(self, cap: int):
        """Edge buffers for at least `cap` edges (a re-run is needed)."""
        if cap <= self.edge_cap:
            return
        self.edge_cap = int(cap)
        self.uv = torch.empty((self.edge_cap, 2), dtype=torch.int32, device=self.device)
        self.bit = torch.empty(self.edge_cap, dtype=torch.int16, device=self.device)
        self._edges_ws()

    def ensure_capacity(self):
        """After a run: grow the edge buffers if they overflowed (needs a re-run)."""
        torch.cuda.synchronize()
        if int(self.status.item()) == B.CG_ECAPACITY:
            self.grow_edges(self.needed_edges())
            return False
        return True

    def host_buffers(self):
        """Pinned host buffers sized to this batch's capacities (for fetch_into)."""
        pin = lambda shape, dt: torch.empty(shape, dtype=dt).pin_memory()
        return {
            "scal": pin(4, torch.int64),
            "cells": pin((max(self.cap_rows, 1), self.words), torch.int32),
            "uv": pin((self.edge_cap, 2), torch.int32),
            "bit": pin(self.edge_cap, torch.int16),
            "offsets": pin(max(self.cap_rows, 1) + 1, torch.int64),
            "r2c": pin(max(self.cap_rows, 1), torch.int32),
            "cell_off": pin(self.cap_scenes + 1, torch.int64),
            "edge_off": pin(self.cap_scenes + 1, torch.int64),
        }

    def fetch_into(self, host, stream):
        """Per-scene results copied through pinned buffers `host` (from
        host_buffers) on `stream`; the returned arrays are views into those
        buffers, valid until they are filled again.  Returns None if the
        edge buffer overflowed (grow_edges, rerun, then fetch again)."""
        with torch.cuda.stream(stream):
            sc = host["scal"]
            sc[0:1].copy_(self.ncells, non_blocking=True)
            sc[1:2].copy_(self.nedges, non_blocking=True)
            sc[2:3].copy_(self.status.to(torch.int64), non_blocking=True)
            k = self.n_scenes + 1
            host["cell_off"][:k].copy_(self.cell_off[:k], non_blocking=True)
            host["edge_off"][:k].copy_(self.edge_off[:k], non_blocking=True)
            host["r2c"][:self.n_rows].copy_(self.r2c[:self.n_rows], non_blocking=True)
            stream.synchronize()
            nc, E, st = int(sc[0]), int(sc[1]), int(sc[2])
            if st != 0:
                return None
            host["cells"][:nc].copy_(self.cells[:nc], non_blocking=True)
            host["uv"][:E].copy_(self.uv[:E], non_blocking=True)
            host["bit"][:E].copy_(self.bit[:E], non_blocking=True)
            host["offsets"][:nc + 1].copy_(self.offsets[:nc + 1], non_blocking=True)
            stream.synchronize()
        cells = host["cells"].numpy().view(np.uint32)
        uv = host["uv"].numpy().view(np.uint32)
        bit = host["bit"].numpy().view(np.uint16)
        off = host["offsets"].numpy()
        r2c = host["r2c"].numpy().view(np.uint32)
        co = host["cell_off"].numpy()
        eo = host["edge_off"].numpy()
        out = []
        for j in range(self.n_scenes):
            wj = -(-int(self.ells[j]) // 32)
            a, b = int(co[j]), int(co[j + 1])
            e0, e1 = int(eo[j]), int(eo[j + 1])
            out.append({
                "ncells": b - a,
                "nedges": e1 - e0,
                "cells": cells[a:b, 1:1 + wj],
                "uv": uv[e0:e1],
                "bit": bit[e0:e1],
                "offsets": off[a:b + 1] - e0,
                "row_to_cell": r2c[self.scene_rows_h[j]:self.scene_rows_h[j + 1]],
            })
        return out

    def fetch(self, sync: bool = True):
        """Per-scene host results: list of dicts (cells in the scene's own u32 layout).
        With sync=False the copies are ordered on the current stream only."""
        if sync:
            torch.cuda.synchronize()
        E = int(self.nedges.item())
        nc = int(self.ncells.item())
        cells = self.cells[:nc].cpu().numpy().view(np.uint32)
        uv = self.uv[:E].cpu().numpy().view(np.uint32)
        bit = self.bit[:E].cpu().numpy().view(np.uint16)
        off = self.offsets[:nc + 1].cpu().numpy()
        r2c = self.r2c[:self.n_rows].cpu().numpy().view(np.uint32)
        co = self.cell_off.cpu().numpy()
        eo = self.edge_off.cpu().numpy()
        out = []
        for j in range(self.n_scenes):
            wj = -(-int(self.ells[j]) // 32)
            a, b = co[j], co[j + 1]
            out.append({
                "ncells": int(b - a),
                "nedges": int(eo[j + 1] - eo[j]),
                "cells": cells[a:b, 1:1 + wj].copy(),
                "uv": uv[eo[j]:eo[j + 1]].copy(),
                "bit": bit[eo[j]:eo[j + 1]].copy(),
                "offsets": off[a:b + 1] - eo[j],
                "row_to_cell": r2c[self.scene_rows_h[j]:self.scene_rows_h[j + 1]].copy(),
            })
        return out


def tuned_params_for(path: str | None = None):
    """params_for(words, rows) for BatchRunner from the autotuner's persisted
    table (tuner.DEFAULT_TABLE unless `path`); classes without an entry get
    the defaults."""
    from . import tuner
    tn = tuner.Tuner(path if path is not None else tuner.DEFAULT_TABLE)
    return lambda words, rows: tn.params_for(words, rows)


class BatchRunner:
    """All classes of a batch; ``run`` launches them on per-class streams,
    ``capture`` records one HIP graph of the whole batch."""

    def __init__(self, shapes, params_for=None, device="cuda"):
        self.shapes = list(shapes)  # (n_j, ell_j)
        groups = {}
        for idx, (n, ell) in enumerate(self.shapes):
            groups.setdefault(class_words(ell), []).append(idx)
        self.classes = []
        for w in sorted(groups):
            ids = groups[w]
            params = params_for(w, sum(self.shapes[i][0] for i in ids)) if params_for else None
            sb = SceneBatch([self.shapes[i][1] for i in ids], [self.shapes[i][0] for i in ids], w, params,
                            device=device)
            self.classes.append((ids, sb))
        self.streams = [torch.cuda.Stream() for _ in self.classes]
        self.graph = None

    def upload(self, scenes):
        for ids, sb in self.classes:
            sb.upload([scenes[i] for i in ids])

    def run(self):
        main = torch.cuda.current_stream()
        for st, (ids, sb) in zip(self.streams, self.classes):
            st.wait_stream(main)
            with torch.cuda.stream(st):
                sb.run(st)
        for st in self.streams:
            main.wait_stream(st)

    def run_checked(self):
        """run(); re-run any class whose edge buffer overflowed, with room."""
        self.run()
        torch.cuda.synchronize()
        again = [sb for _, sb in self.classes if not sb.ensure_capacity()]
        for sb in again:
            sb.run()
        torch.cuda.synchronize()

    def capture(self):
        """Record the whole batch (all classes, their streams) into one graph."""
        self.graph = torch.cuda.CUDAGraph()
        cap_stream = torch.cuda.Stream()
        cap_stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=cap_stream):
            self.run()
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()

    def fetch(self):
        res = [None] * len(self.shapes)
        for ids, sb in self.classes:
            for i, r in zip(ids, sb.fetch()):
                res[i] = r
        return res

    def totals(self):
        torch.cuda.synchronize()
        return (sum(int(sb.ncells.item()) for _, sb in self.classes),
                sum(int(sb.nedges.item()) for _, sb in self.classes))
