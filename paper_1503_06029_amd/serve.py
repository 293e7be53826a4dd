"""Serving loop: continuous batching of cell-graph requests.

Requests (arrival time, scene) are admitted into the next batch as soon as
they have arrived and the batch has room: each width class has a fixed
device footprint (rows, scenes, sign bytes, edges), and a request that does
not fit waits for the next batch.  Two batch slots alternate: while one
batch computes on its stream, the host admits the next arrivals, copies
their sign bytes (request payloads held in pinned host memory) straight into
the other slot's device buffer and launches it, then collects the finished
batch through pinned result buffers.  So requests that arrive while others are on
the GPU are picked up as soon as a slot frees, and copies of one batch
overlap the compute of the other.  Latency is measured from a request's
arrival to the moment its results are on the host.

Dictionaries stay resident: after a scene's first batch its cells,
row_to_cell and dictionary are kept on the device (ResidentPool, an LRU
within a byte budget taken from the free device memory), and a later request
for that scene recomputes its edges from the resident dictionary with
cg_edges instead of packing, deduplicating and building again.

Every request ends with a result whose "status" is "ok", "rejected" (no
batch can hold it), "cancelled" (cancelled before its result was
delivered) or "error" (a device allocation or library call failed for its
batch; the loop goes on with the other requests).

The per-scene baseline serves the same trace one request at a time with
plain per-scene launches (preallocated per pool scene).

Only scheduling, staging and marshalling live here; all compute is in the
library's kernels.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque

import numpy as np
import torch

from . import batch as BT
from . import pipeline


from . import binding as B

# Host staging of one slot's resident-scene results (pinned): rows of
# row_to_cell, cell words, edges and offsets per batch.  A resident request
# is admitted into a batch while its results fit what is left of these.
STAGE_CAPS = (1 << 22, 1 << 23, 1 << 22, 1 << 22, 4096)  # ..., and distinct scenes


def resident_footprint(ncells: int, n_rows: int, ell: int) -> int:
    """Device bytes one resident scene holds: its cells (ceil(l / 32) uint32
    words each), row_to_cell, cell count and dictionary memory (the size
    cg_dict_size reports)."""
    lay = B.make_layout(ell, 32)
    nc = max(int(ncells), 1)
    return 4 * nc * lay.words + 4 * max(int(n_rows), 1) + 8 + B.cg_dict_size(nc, lay, None)


def _torch_alloc(shape, dtype, device):
    return torch.empty(shape, dtype=dtype, device=device)


class ResidentScene:
    """One scene's dictionary kept on the device between requests: its
    sorted cells (uint32 words, its own layout), row_to_cell and dictionary
    memory; the dictionary borrows the cells.  Built once from a batch's
    output slice; read-only afterwards."""

    def __init__(self, si: int, ell: int, n_rows: int, ncells: int, nedges: int, device, alloc=_torch_alloc):
        self.si, self.ell, self.n_rows, self.ncells, self.nedges = si, int(ell), int(n_rows), int(ncells), int(nedges)
        self.lay = B.make_layout(self.ell, 32)
        nc = max(self.ncells, 1)
        self.cells = alloc((nc, self.lay.words), torch.int32, device)
        self.r2c = alloc((max(self.n_rows, 1),), torch.int32, device)
        self.ncells_dev = alloc((1,), torch.int64, device)
        self.dict_bytes = B.cg_dict_size(nc, self.lay, None)
        self.dict_mem = alloc((self.dict_bytes,), torch.uint8, device)
        self.bytes = resident_footprint(self.ncells, self.n_rows, self.ell)
        self.dict = None
        self.ready = None   # event recorded after the build
        self.users = 0      # in-flight batches reading it (never evicted while > 0)

    def build(self, sb, a: int, r0: int, stream):
        """Copy the scene's cells (words 1.. of its virtual rows a .. a +
        ncells of class batch sb) and row_to_cell, then cg_dict_build, all on
        `stream` (ordered before the batch buffers are reused)."""
        wj = self.lay.words
        with torch.cuda.stream(stream):
            if self.ncells:
                self.cells[:self.ncells].copy_(sb.cells[a:a + self.ncells, 1:1 + wj])
            if self.n_rows:
                self.r2c[:self.n_rows].copy_(sb.r2c[r0:r0 + self.n_rows])
            self.ncells_dev.fill_(self.ncells)
            self.dict = B.cg_dict_build(self.cells, self.ncells_dev, max(self.ncells, 1), self.lay, None,
                                        self.dict_mem, self.dict_bytes, stream)
            self.ready = torch.cuda.Event()
            self.ready.record(stream)

    def stage_need(self):
        """(rows, cell words, edges, offsets, scenes) of host staging its result takes."""
        return (self.n_rows, self.ncells * self.lay.words, self.nedges, self.ncells + 1, 1)


class ResidentPool:
    """LRU of resident scene dictionaries within `budget` device bytes.
    Scenes in use by an in-flight batch are never evicted; a scene that does
    not fit, or whose buffers cannot be allocated, simply stays non-resident
    (its requests go through the batched path)."""

    def __init__(self, budget: int, device="cuda", alloc=_torch_alloc):
        self.budget = int(budget)
        self.device = device
        self.alloc = alloc
        self.scenes: OrderedDict[int, ResidentScene] = OrderedDict()
        self.used = 0
        self.hits = self.misses = self.evictions = self.alloc_failures = 0

    def get(self, si: int):
        e = self.scenes.get(si)
        if e is not None:
            self.scenes.move_to_end(si)
        return e

    def _make_room(self, need: int) -> bool:
        if need > self.budget:
            return False
        for si in list(self.scenes):
            if self.used + need <= self.budget:
                break
            e = self.scenes[si]
            if e.users == 0:
                del self.scenes[si]
                self.used -= e.bytes
                self.evictions += 1
        return self.used + need <= self.budget

    def add(self, si: int, ell: int, n_rows: int, ncells: int, nedges: int, sb, a: int, r0: int, stream) -> bool:
        """Make scene si resident from its slice of class batch sb (cells from
        virtual cell a, rows from virtual row r0).  Returns whether it is."""
        if si in self.scenes or self.budget <= 0:
            return si in self.scenes
        if not self._make_room(resident_footprint(ncells, n_rows, ell)):
            return False
        try:
            # allocated on the building stream: once evicted, the memory is only
            # reused by later work on that stream, after the build
            with torch.cuda.stream(stream):
                e = ResidentScene(si, ell, n_rows, ncells, nedges, self.device, self.alloc)
            e.build(sb, a, r0, stream)
        except (torch.cuda.OutOfMemoryError, MemoryError, B.CellGraphError):
            self.alloc_failures += 1
            return False
        self.scenes[si] = e
        self.used += e.bytes
        return True


class Slot:
    """Device buffers for one in-flight batch (one SceneBatch per class), the
    device outputs of edges recomputed from resident dictionaries, and the
    pinned host buffers results come back through."""

    def __init__(self, class_caps, device="cuda", stage_caps=STAGE_CAPS):
        self.stream = torch.cuda.Stream()
        self.device = device
        self.batches = {}
        self.host = {}
        for w, (rows, scenes, nbytes) in class_caps.items():
            ell = 32 * (w - 1)
            sb = BT.SceneBatch([ell], [1], w, max_rows=rows, max_scenes=scenes, max_bytes=nbytes,
                               edge_cap=max(4096, 4 * rows), device=device)
            self.batches[w] = sb
            self.host[w] = sb.host_buffers()
        self.stage_caps = tuple(int(c) for c in stage_caps)
        self.stage = None        # pinned staging of resident results, made on first use
        self.rdev = None         # device outputs for resident edges: (ncells cap, edge cap) and buffers
        self.requests = None
        self.resident_reqs = None
        self.done = None

    # ------------------------------------------------ resident dictionaries
    def _stage_buffers(self):
        if self.stage is None:
            rows, cw, edges, offs, nsc = self.stage_caps
            pin = lambda shape, dt: torch.empty(shape, dtype=dt).pin_memory()
            self.stage = {"r2c": pin(rows, torch.int32), "cells": pin(cw, torch.int32),
                          "uv": pin((edges, 2), torch.int32), "bit": pin(edges, torch.int16),
                          "offsets": pin(offs, torch.int64), "scal": pin((nsc, 2), torch.int64)}
        return self.stage

    def _resident_outputs(self, e: ResidentScene):
        """Device edge outputs and workspace big enough for resident scene e
        (grown, on this slot's stream, when a larger scene comes)."""
        nc, E = max(e.ncells, 1), max(e.nedges, 1)
        r = self.rdev
        ws = B.cg_edges_workspace(e.dict, E)
        if r is None or nc > r["nc"] or E > r["E"] or ws > r["ws_bytes"]:
            nc = max(nc, r["nc"] if r else 0)
            E = max(E, r["E"] if r else 0)
            ws = max(ws, r["ws_bytes"] if r else 0)
            dev = self.device
            r = {"nc": nc, "E": E, "ws_bytes": ws,
                 "uv": torch.empty((E, 2), dtype=torch.int32, device=dev),
                 "bit": torch.empty(E, dtype=torch.int16, device=dev),
                 "offsets": torch.empty(nc + 1, dtype=torch.int64, device=dev),
                 "scal": torch.zeros(2, dtype=torch.int64, device=dev),
                 "status": torch.zeros(1, dtype=torch.int32, device=dev),
                 "ws": torch.empty(ws, dtype=torch.uint8, device=dev)}
            self.rdev = r
        return r

    def _launch_resident(self, reqs, pool: ResidentPool):
        """Edges of resident scenes from their dictionaries, one cg_edges per
        distinct scene of the batch, each followed by its copies into the
        pinned staging (stream order keeps the shared device outputs safe)."""
        st = self._stage_buffers()
        plan = {}
        o = [0, 0, 0, 0]
        self.resident_reqs = (list(reqs), plan)  # held scenes are released on collect or release()
        for rid, si in reqs:
            if si in plan:
                continue
            e = pool.get(si)
            e.users += 1
            rows, cw, edges, offs, _ = e.stage_need()
            plan[si] = (e, tuple(o), len(plan))
            o = [o[0] + rows, o[1] + cw, o[2] + edges, o[3] + offs]
        for si, (e, (r0, c0, e0, f0), k) in plan.items():
            self.stream.wait_event(e.ready)
            r = self._resident_outputs(e)
            B.cg_edges(e.dict, r["uv"], r["bit"], r["E"], r["scal"][0:1], r["offsets"], r["ws"], r["ws_bytes"],
                       r["status"], self.stream)
            r["scal"][1:2].copy_(r["status"].to(torch.int64))
            nc, E, W = e.ncells, e.nedges, e.lay.words
            st["scal"][k].copy_(r["scal"], non_blocking=True)
            if E:
                st["uv"][e0:e0 + E].copy_(r["uv"][:E], non_blocking=True)
                st["bit"][e0:e0 + E].copy_(r["bit"][:E], non_blocking=True)
            st["offsets"][f0:f0 + nc + 1].copy_(r["offsets"][:nc + 1], non_blocking=True)
            if nc:
                st["cells"][c0:c0 + nc * W].copy_(e.cells[:nc].reshape(-1), non_blocking=True)
            if e.n_rows:
                st["r2c"][r0:r0 + e.n_rows].copy_(e.r2c[:e.n_rows], non_blocking=True)

    def _collect_resident(self, copy: bool):
        reqs, plan = self.resident_reqs
        st = self.stage
        scal = st["scal"].numpy()
        by_scene = {}
        for si, (e, (r0, c0, e0, f0), k) in plan.items():
            e.users -= 1
            nc, E, W = e.ncells, e.nedges, e.lay.words
            if int(scal[k, 0]) != E or int(scal[k, 1]) != 0:
                by_scene[si] = {"status": "error",
                                "reason": f"resident scene {si}: {int(scal[k, 0])} edges (status {int(scal[k, 1])}), "
                                          f"expected {E}"}
                continue
            res = {"ncells": nc, "nedges": E,
                   "cells": st["cells"].numpy().view(np.uint32)[c0:c0 + nc * W].reshape(nc, W),
                   "uv": st["uv"].numpy().view(np.uint32)[e0:e0 + E],
                   "bit": st["bit"].numpy().view(np.uint16)[e0:e0 + E],
                   "offsets": st["offsets"].numpy()[f0:f0 + nc + 1],
                   "row_to_cell": st["r2c"].numpy().view(np.uint32)[r0:r0 + e.n_rows],
                   "status": "ok", "resident": True}
            by_scene[si] = res
        out = {}
        for rid, si in reqs:
            r = by_scene[si]
            out[rid] = {k: (v.copy() if copy and isinstance(v, np.ndarray) else v) for k, v in r.items()}
        self.resident_reqs = None
        return out

    # ------------------------------------------------------------- batches
    def launch(self, reqs, scenes, pinned, resident=(), pool=None):
        """Copy and launch one batch: reqs = [(req_id, scene_idx)]; pinned[si]
        is scene si's sign bytes in pinned host memory (one copy per request,
        straight into the batch's device buffer).  `resident` requests
        [(req_id, scene_idx)] name scenes resident in `pool`: their edges are
        recomputed from the resident dictionaries on the same stream."""
        by_class = {}
        for rid, si in reqs:
            R = scenes[si]
            by_class.setdefault(BT.class_words(R.shape[1]), []).append((rid, si))
        self.requests = by_class
        self.resident_reqs = None
        with torch.cuda.stream(self.stream):
            for w, items in by_class.items():
                sb = self.batches[w]
                sb.set_scenes([scenes[si].shape[1] for _, si in items], [scenes[si].shape[0] for _, si in items])
                o = 0
                for _, si in items:
                    m = pinned[si].numel()
                    if m:
                        sb.bits[o:o + m].copy_(pinned[si], non_blocking=True)
                    o += m
                sb.run(self.stream)
            if resident:
                self._launch_resident(resident, pool)
            self.done = torch.cuda.Event()
            self.done.record(self.stream)

    def launch_sampled(self, reqs, descs, planes, plane_off, box, resident=(), pool=None):
        """Launch one batch of sampled scenes: descs[si] = (planes, n, key);
        the scenes' planes sit in the device pool `planes` from plane_off[si].
        Only the scene table (offsets, sizes, keys) crosses PCIe."""
        by_class = {}
        for rid, si in reqs:
            ell = descs[si][0].shape[0]
            by_class.setdefault(BT.class_words(ell), []).append((rid, si))
        self.requests = by_class
        self.resident_reqs = None
        with torch.cuda.stream(self.stream):
            for w, items in by_class.items():
                sb = self.batches[w]
                sb.set_sampled([descs[si][0].shape[0] for _, si in items], [descs[si][1] for _, si in items],
                               [plane_off[si] for _, si in items], [descs[si][2] for _, si in items])
                sb.run_sampled(planes, box, self.stream)
            if resident:
                self._launch_resident(resident, pool)
            self.done = torch.cuda.Event()
            self.done.record(self.stream)

    def request_ids(self):
        """Ids of the requests of the launched batch (batched and resident)."""
        ids = [rid for items in (self.requests or {}).values() for rid, _ in items]
        return ids + [rid for rid, _ in (self.resident_reqs[0] if self.resident_reqs else [])]

    def release(self):
        """After a failed launch or collect: wait for whatever was enqueued, drop the
        batch and release the resident scenes it held."""
        self.stream.synchronize()
        if self.resident_reqs is not None:
            for e, _, _ in self.resident_reqs[1].values():
                e.users -= 1
        self.requests = None
        self.resident_reqs = None

    def collect(self, copy: bool = False, pool: ResidentPool | None = None):
        """Wait for the batch; return {req_id: result dict}.  Copies go on the
        slot's own stream, so the other slot's batch keeps running.  Results
        are views into this slot's pinned buffers (valid until the slot runs
        again) unless copy=True.  A class whose edges overflowed its edge
        buffer is grown and run again (its inputs are still in place), so
        every request gets its exact result; each result has "status": "ok".
        With a pool, scenes of the batch that are not yet resident are made
        resident from the batch's output (enqueued here, before the slot's
        buffers can be reused)."""
        self.done.synchronize()
        out = {}
        for w, items in self.requests.items():
            sb = self.batches[w]
            res = sb.fetch_into(self.host[w], self.stream)
            if res is None:
                with torch.cuda.stream(self.stream):
                    sb.grow_edges(sb.needed_edges())
                    self.host[w] = sb.host_buffers()
                    sb.rerun(self.stream)
                self.stream.synchronize()
                res = sb.fetch_into(self.host[w], self.stream)
                assert res is not None
            co = self.host[w]["cell_off"].numpy()
            for j, ((rid, si), r) in enumerate(zip(items, res)):
                out[rid] = {k: (v.copy() if copy and isinstance(v, np.ndarray) else v) for k, v in r.items()}
                out[rid]["status"] = "ok"
                if pool is not None and pool.get(si) is None:
                    ok = pool.add(si, int(sb.ells[j]), int(sb.ns[j]), r["ncells"], r["nedges"], sb, int(co[j]),
                                  int(sb.scene_rows_h[j]), self.stream)
                    pool.misses += 1
                    if ok:
                        out[rid]["made_resident"] = True
        if self.resident_reqs is not None:
            res = self._collect_resident(copy)
            if pool is not None:
                pool.hits += len(res)
            out.update(res)
        self.requests = None
        return out


def admit_requests(queue: deque, now: float, caps, shapes, resident=None, stage=STAGE_CAPS):
    """Take the requests that have arrived by `now`, in arrival order, while
    their width class has room (rows, scenes, sign bytes); the others stay
    queued, still in arrival order.  queue holds (req_id, arrival, scene);
    shapes[scene] = (rows, l).

    A request that no batch can ever hold (its l is longer than any width
    class, its class has no capacity here, or its rows or sign bytes alone
    exceed the class's capacity) is taken off the queue and rejected, so it
    never blocks the loop.

    With `resident` (scene -> its staging need (rows, cell words, edges,
    offsets) if its dictionary is resident, else None), requests for
    resident scenes take no class capacity, only host staging (`stage`,
    the same four quantities); they are returned apart.

    Returns (taken [(req_id, scene)], rejected [(req_id, scene, reason)]),
    and, with `resident`, also the resident requests [(req_id, scene)]."""
    used = {w: [0, 0, 0] for w in caps}
    staged = [0] * len(stage)
    taken, rejected, res_taken = [], [], []
    keep = deque()
    while queue and queue[0][1] <= now:
        rid, t, si = queue.popleft()
        n, ell = shapes[si]
        need = resident(si) if resident is not None else None
        if need is not None and all(x <= c for x, c in zip(need, stage)):
            if all(u + x <= c for u, x, c in zip(staged, need, stage)):
                staged = [u + x for u, x in zip(staged, need)]
                res_taken.append((rid, si))
            else:
                keep.append((rid, t, si))  # staging full: the next batch
            continue
        reason = None
        try:
            w = BT.class_words(ell)
        except ValueError:
            w = None
            reason = f"l = {ell} is longer than any batch class"
        if w is not None and w not in caps:
            reason = f"no capacity for {w}-word rows"
        if reason is None:
            rows, nsc, nb = caps[w]
            if n > rows or n * ell > nb or nsc < 1:
                reason = f"{n} rows of l = {ell} exceed the batch footprint ({rows} rows, {nb} sign bytes)"
        if reason is not None:
            rejected.append((rid, si, reason))
            continue
        u = used[w]
        if u[0] + n <= rows and u[1] + 1 <= nsc and u[2] + n * ell <= nb:
            u[0] += n
            u[1] += 1
            u[2] += n * ell
            taken.append((rid, si))
        else:
            keep.append((rid, t, si))  # no room in this batch: the next one
    keep.extend(queue)  # skipped requests arrived first: order is kept
    queue.clear()
    queue.extend(keep)
    if resident is not None:
        return taken, rejected, res_taken
    return taken, rejected


def plan_capacity(class_words, free_bytes: int, fraction: float = 0.5, slots: int = 2,
                  max_rows: int = 1 << 21, scenes_per_class: int = 4096):
    """Rows per width class so that `slots` batch slots, each holding one
    batch of every class at that capacity, fit in `fraction` of `free_bytes`
    of device memory (the device footprint of a class batch, from the
    library's workspace sizes, is batch.class_footprint).  Returns (rows,
    footprint in bytes of all slots)."""
    budget = int(free_bytes * fraction)
    rows = max_rows
    while rows > 1024:
        tot = slots * sum(BT.class_footprint(rows, scenes_per_class, rows * 32 * (w - 1), w)
                          for w in class_words)
        if tot <= budget:
            return rows, tot
        rows //= 2
    tot = slots * sum(BT.class_footprint(rows, scenes_per_class, rows * 32 * (w - 1), w) for w in class_words)
    return rows, tot


_FAILURES = (torch.cuda.OutOfMemoryError, MemoryError, B.CellGraphError)


class Server:
    """Continuous batching over a pool of scenes given as sign bytes.

    Class capacities: `rows_per_class` rows (and 32 (w - 1) sign bytes per
    row) per width class w, or, with rows_per_class=None, the largest power
    of two whose two slots fit in half of the device memory that is free
    when the server starts (plan_capacity).  `resident_fraction` of the
    device memory free after the slots are made (torch.cuda.mem_get_info) is
    the resident-dictionary budget; 0 turns resident dictionaries off."""

    def __init__(self, scenes, rows_per_class: int | None = 1 << 21, scenes_per_class: int = 4096,
                 device="cuda", resident_fraction: float = 0.25, resident_budget: int | None = None):
        self.scenes = scenes
        self.shapes = [R.shape for R in scenes]
        ells = sorted({BT.class_words(R.shape[1]) for R in scenes if R.shape[1] <= BT.MAX_ELL})
        if rows_per_class is None:
            free, _ = torch.cuda.mem_get_info()
            rows_per_class, self.footprint = plan_capacity(ells, free, scenes_per_class=scenes_per_class)
        caps = {}
        for w in ells:
            caps[w] = (rows_per_class, scenes_per_class, rows_per_class * 32 * (w - 1))
        self.caps = caps
        self.slots = [Slot(caps, device), Slot(caps, device)]
        # the request payloads (sign bytes) live in pinned host memory
        self.pinned = [torch.from_numpy(np.ascontiguousarray(R, dtype=np.uint8).reshape(-1)).pin_memory()
                       for R in scenes]
        self.pool = self._make_pool(device, resident_fraction, resident_budget)

    @staticmethod
    def _make_pool(device, fraction, budget):
        if budget is None:
            budget = int(torch.cuda.mem_get_info()[0] * fraction) if fraction > 0 else 0
        return ResidentPool(budget, device) if budget > 0 else None

    def _resident_need(self, si):
        e = self.pool.get(si) if self.pool is not None else None
        return e.stage_need() if e is not None else None

    def _admit(self, queue: deque, now: float):
        return admit_requests(queue, now, self.caps, self.shapes, resident=self._resident_need)

    def _launch(self, slot, reqs, res_reqs):
        slot.launch(reqs, self.scenes, self.pinned, res_reqs, self.pool)

    def serve(self, arrivals, scene_idx, keep_results: bool = False, sink=None, cancels=None):
        """Serve a trace in real time.  Returns (latencies in s, results or
        None, wall seconds).  Every request ends with one result, whose
        "status" is "ok", "rejected" (with a "reason") for a request no batch
        can hold, "cancelled", or "error" (with a "reason") when its batch
        could not be launched or collected; rejected and cancelled requests
        are answered at once.  cancels: (time, req_id) pairs; a request
        cancelled before its result is delivered is answered "cancelled"
        (queued: taken off the queue; in flight: its result is dropped).
        sink(req_id, result), if given, sees every result as it arrives (its
        arrays are views that stay valid only during the call)."""
        n = len(arrivals)
        queue = deque((i, float(arrivals[i]), int(scene_idx[i])) for i in range(n))
        cq = deque(sorted((float(t), int(r)) for t, r in (cancels if cancels is not None else ())))
        lat = np.zeros(n)
        results = {} if keep_results else None
        self.rejected, self.errors, self.cancelled = [], [], []
        answered = np.zeros(n, dtype=bool)
        to_cancel = set()
        inflight = []  # slots with a launched batch, oldest first
        free = list(self.slots)
        t0 = time.perf_counter()

        def answer(rid, r, tnow):
            lat[rid] = tnow - arrivals[rid]
            answered[rid] = True
            if keep_results:
                results[rid] = r
            if sink is not None:
                sink(rid, r)

        served = 0
        while served < n:
            now = time.perf_counter() - t0
            progressed = False
            while cq and cq[0][0] <= now:
                _, rid = cq.popleft()
                if answered[rid]:
                    continue
                for k, item in enumerate(queue):
                    if item[0] == rid:
                        del queue[k]
                        self.cancelled.append(rid)
                        answer(rid, {"status": "cancelled"}, now)
                        served += 1
                        break
                else:
                    to_cancel.add(rid)  # in flight (or not yet arrived): dropped when it completes
                progressed = True
            if free and queue and queue[0][1] <= now:
                reqs, rej, res_reqs = self._admit(queue, now)
                tnow = time.perf_counter() - t0
                for rid, si, why in rej:
                    self.rejected.append(rid)
                    answer(rid, {"status": "rejected", "reason": why}, tnow)
                served += len(rej)
                progressed = bool(rej)
                if reqs or res_reqs:
                    slot = free.pop(0)
                    try:
                        self._launch(slot, reqs, res_reqs)
                        inflight.append(slot)
                    except _FAILURES as exc:
                        slot.release()
                        free.append(slot)
                        tnow = time.perf_counter() - t0
                        for rid, _ in list(reqs) + list(res_reqs):
                            self.errors.append(rid)
                            answer(rid, {"status": "error", "reason": f"launch: {exc}"}, tnow)
                        served += len(reqs) + len(res_reqs)
                    progressed = True
            if inflight and (not free or inflight[0].done.query()):
                slot = inflight.pop(0)
                try:
                    out = slot.collect(copy=keep_results, pool=self.pool)
                except _FAILURES as exc:
                    ids = slot.request_ids()
                    slot.release()
                    out = {rid: {"status": "error", "reason": f"collect: {exc}"} for rid in ids}
                    self.errors.extend(ids)
                tdone = time.perf_counter() - t0
                for rid, r in out.items():
                    if rid in to_cancel:
                        self.cancelled.append(rid)
                        r = {"status": "cancelled"}
                    answer(rid, r, tdone)
                served += len(out)
                free.append(slot)
                progressed = True
            if not progressed:
                wait = (queue[0][1] - (time.perf_counter() - t0)) if queue else 0.0002
                time.sleep(min(max(wait, 0.0), 0.0002))
        wall = time.perf_counter() - t0
        return lat, results, wall


class SampledServer(Server):
    """The same continuous batching with scenes given as descriptions
    (planes, points, generator key) and sampled on the GPU: a request moves
    a few bytes of scene table instead of its sign bytes."""

    def __init__(self, descs, box, rows_per_class: int = 1 << 21, scenes_per_class: int = 4096, device="cuda",
                 resident_fraction: float = 0.25, resident_budget: int | None = None):
        self.descs = descs
        self.box = box
        caps, slot_caps = {}, {}
        for pl, n, key in descs:
            w = BT.class_words(pl.shape[0])
            caps[w] = (rows_per_class, scenes_per_class, 1 << 62)  # no sign bytes to hold
            slot_caps[w] = (rows_per_class, scenes_per_class, 4096)
        self.caps = caps
        self.slots = [Slot(slot_caps, device), Slot(slot_caps, device)]
        off = np.zeros(len(descs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([d[0].shape[0] for d in descs])
        self.plane_off = off
        self.planes = torch.from_numpy(np.concatenate([d[0] for d in descs]).astype(np.float64)).to(device)
        self.shapes = [(d[1], d[0].shape[0]) for d in descs]
        self.pool = self._make_pool(device, resident_fraction, resident_budget)

    def _launch(self, slot, reqs, res_reqs):
        slot.launch_sampled(reqs, self.descs, self.planes, self.plane_off, self.box, res_reqs, self.pool)


class PerSceneBaseline:
    """The same trace with plain per-scene launches, one request at a time."""

    def __init__(self, scenes, device="cuda"):
        self.scenes = scenes
        self.graphs = {}
        self.bits = {}
        for si, R in enumerate(scenes):
            g = pipeline.CellGraph(R.shape[0], R.shape[1], 32, edge_cap=max(4096, 4 * R.shape[0]),
                                   device=device)
            self.graphs[si] = g
            self.bits[si] = torch.from_numpy(np.ascontiguousarray(R)).pin_memory()
        self.dev_bits = {}

    def serve(self, arrivals, scene_idx, keep_results: bool = False):
        n = len(arrivals)
        lat = np.zeros(n)
        results = {} if keep_results else None
        t0 = time.perf_counter()
        for i in range(n):
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            si = int(scene_idx[i])
            g = self.graphs[si]
            R = self.scenes[si]
            dev = torch.empty(R.shape, dtype=torch.uint8, device="cuda")
            dev.copy_(self.bits[si], non_blocking=True)
            if R.shape[0]:
                g.pack(dev)
            g.run()
            r = g.fetch()
            lat[i] = time.perf_counter() - t0 - arrivals[i]
            if keep_results:
                results[i] = r
        wall = time.perf_counter() - t0
        return lat, results, wall
