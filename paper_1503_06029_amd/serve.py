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

The per-scene baseline serves the same trace one request at a time with
plain per-scene launches (preallocated per pool scene).

Only scheduling, staging and marshalling live here; all compute is in the
library's kernels.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np
import torch

from . import batch as BT
from . import pipeline


class Slot:
    """Device buffers for one in-flight batch (one SceneBatch per class) and
    the pinned host buffers its results come back through."""

    def __init__(self, class_caps, device="cuda"):
        self.stream = torch.cuda.Stream()
        self.batches = {}
        self.host = {}
        for w, (rows, scenes, nbytes) in class_caps.items():
            ell = 32 * (w - 1)
            sb = BT.SceneBatch([ell], [1], w, max_rows=rows, max_scenes=scenes, max_bytes=nbytes,
                               edge_cap=max(4096, 4 * rows), device=device)
            self.batches[w] = sb
            self.host[w] = sb.host_buffers()
        self.requests = None
        self.done = None

    def launch(self, reqs, scenes, pinned):
        """Copy and launch one batch: reqs = [(req_id, scene_idx)]; pinned[si]
        is scene si's sign bytes in pinned host memory (one copy per request,
        straight into the batch's device buffer)."""
        by_class = {}
        for rid, si in reqs:
            R = scenes[si]
            by_class.setdefault(BT.class_words(R.shape[1]), []).append((rid, si))
        self.requests = by_class
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
            self.done = torch.cuda.Event()
            self.done.record(self.stream)

    def launch_sampled(self, reqs, descs, planes, plane_off, box):
        """Launch one batch of sampled scenes: descs[si] = (planes, n, key);
        the scenes' planes sit in the device pool `planes` from plane_off[si].
        Only the scene table (offsets, sizes, keys) crosses PCIe."""
        by_class = {}
        for rid, si in reqs:
            ell = descs[si][0].shape[0]
            by_class.setdefault(BT.class_words(ell), []).append((rid, si))
        self.requests = by_class
        with torch.cuda.stream(self.stream):
            for w, items in by_class.items():
                sb = self.batches[w]
                sb.set_sampled([descs[si][0].shape[0] for _, si in items], [descs[si][1] for _, si in items],
                               [plane_off[si] for _, si in items], [descs[si][2] for _, si in items])
                sb.run_sampled(planes, box, self.stream)
            self.done = torch.cuda.Event()
            self.done.record(self.stream)

    def collect(self, copy: bool = False):
        """Wait for the batch; return {req_id: result dict}.  Copies go on the
        slot's own stream, so the other slot's batch keeps running.  Results
        are views into this slot's pinned buffers (valid until the slot runs
        again) unless copy=True.  A class whose edges overflowed its edge
        buffer is grown and run again (its inputs are still in place), so
        every request gets its exact result; each result has "status": "ok"."""
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
            for (rid, _), r in zip(items, res):
                out[rid] = {k: (v.copy() if copy and isinstance(v, np.ndarray) else v) for k, v in r.items()}
                out[rid]["status"] = "ok"
        self.requests = None
        return out


def admit_requests(queue: deque, now: float, caps, shapes):
    """Take the requests that have arrived by `now`, in arrival order, while
    their width class has room (rows, scenes, sign bytes); the others stay
    queued, still in arrival order.  queue holds (req_id, arrival, scene);
    shapes[scene] = (rows, l).

    A request that no batch can ever hold (its l is longer than any width
    class, its class has no capacity here, or its rows or sign bytes alone
    exceed the class's capacity) is taken off the queue and rejected, so it
    never blocks the loop.  Returns (taken [(req_id, scene)], rejected
    [(req_id, scene, reason)])."""
    used = {w: [0, 0, 0] for w in caps}
    taken, rejected = [], []
    keep = deque()
    while queue and queue[0][1] <= now:
        rid, t, si = queue.popleft()
        n, ell = shapes[si]
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


class Server:
    """Continuous batching over a pool of scenes given as sign bytes.

    Class capacities: `rows_per_class` rows (and 32 (w - 1) sign bytes per
    row) per width class w, or, with rows_per_class=None, the largest power
    of two whose two slots fit in half of the device memory that is free
    when the server starts (plan_capacity)."""

    def __init__(self, scenes, rows_per_class: int | None = 1 << 21, scenes_per_class: int = 4096,
                 device="cuda"):
        self.scenes = scenes
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

    def _admit(self, queue: deque, now: float):
        return admit_requests(queue, now, self.caps, [R.shape for R in self.scenes])

    def _launch(self, slot, reqs):
        slot.launch(reqs, self.scenes, self.pinned)

    def serve(self, arrivals, scene_idx, keep_results: bool = False, sink=None):
        """Serve a trace in real time.  Returns (latencies in s, results or
        None, wall seconds).  Every request ends with a result whose "status"
        is "ok", or "rejected" (with a "reason") for a request no batch can
        hold; rejected requests are answered at once.  sink(req_id, result),
        if given, sees every result as it arrives (its arrays are views that
        stay valid only during the call)."""
        n = len(arrivals)
        queue = deque((i, float(arrivals[i]), int(scene_idx[i])) for i in range(n))
        lat = np.zeros(n)
        results = {} if keep_results else None
        self.rejected = []
        inflight = []  # slots with a launched batch, oldest first
        free = list(self.slots)
        t0 = time.perf_counter()
        served = 0
        while served < n:
            now = time.perf_counter() - t0
            progressed = False
            if free and queue and queue[0][1] <= now:
                reqs, rej = self._admit(queue, now)
                tnow = time.perf_counter() - t0
                for rid, si, why in rej:
                    lat[rid] = tnow - arrivals[rid]
                    self.rejected.append(rid)
                    r = {"status": "rejected", "reason": why}
                    if keep_results:
                        results[rid] = r
                    if sink is not None:
                        sink(rid, r)
                served += len(rej)
                progressed = bool(rej)
                if reqs:
                    slot = free.pop(0)
                    self._launch(slot, reqs)
                    inflight.append(slot)
                    progressed = True
            if inflight and (not free or inflight[0].done.query()):
                slot = inflight.pop(0)
                out = slot.collect(copy=keep_results)
                tdone = time.perf_counter() - t0
                for rid, r in out.items():
                    lat[rid] = tdone - arrivals[rid]
                    if keep_results:
                        results[rid] = r
                    if sink is not None:
                        sink(rid, r)
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

    def __init__(self, descs, box, rows_per_class: int = 1 << 21, scenes_per_class: int = 4096, device="cuda"):
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

    def _admit(self, queue: deque, now: float):
        return admit_requests(queue, now, self.caps, self.shapes)

    def _launch(self, slot, reqs):
        slot.launch_sampled(reqs, self.descs, self.planes, self.plane_off, self.box)


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
