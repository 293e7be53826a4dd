"""Admission logic and termination of the serving loop, on the CPU (no device work)."""
from collections import deque

import numpy as np
import torch

from paper_1503_06029_amd import serve
from paper_1503_06029_amd.batch import class_words, class_footprint, CLASS_WORDS


def test_class_words():
    assert [class_words(l) for l in (1, 32, 33, 96, 97, 224, 225, 480, 481, 992)] == [2, 2, 4, 4, 8, 8, 16, 16, 32, 32]


def test_admission_respects_arrival_and_capacity():
    shapes = [(100, 20), (300, 20), (50, 200), (400, 20)]
    caps = {2: (500, 8, 500 * 32), 8: (100, 2, 100 * 224)}
    q = deque([(0, 0.0, 0), (1, 0.1, 1), (2, 0.2, 2), (3, 0.3, 3), (4, 5.0, 0)])
    taken, rej = serve.admit_requests(q, 1.0, caps, shapes)
    # request 3 (400 rows) does not fit after 0 and 1 (400 of 500 rows used); 4 has not arrived
    assert taken == [(0, 0), (1, 1), (2, 2)] and rej == []
    assert [r[0] for r in q] == [3, 4]
    taken, rej = serve.admit_requests(q, 1.0, caps, shapes)
    assert taken == [(3, 3)] and [r[0] for r in q] == [4]
    assert serve.admit_requests(q, 1.0, caps, shapes) == ([], [])
    assert serve.admit_requests(q, 6.0, caps, shapes) == ([(4, 0)], [])


def test_admission_scene_limit_and_no_starvation():
    shapes = [(1, 10)]
    caps = {2: (1000, 3, 1000 * 32)}
    q = deque((i, 0.0, 0) for i in range(10))
    rounds = []
    while q:
        rounds.append([r for r, _ in serve.admit_requests(q, 0.0, caps, shapes)[0]])
    assert rounds == [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9]]


def test_oversized_requests_are_rejected_not_requeued():
    # scene 1 has more rows than its class holds, scene 2 is longer than any
    # class, scene 3's class has no capacity: each is rejected at once, and
    # requests behind them are still admitted in order
    shapes = [(100, 20), (500, 20), (10, 5000), (10, 100)]
    caps = {2: (200, 8, 200 * 32)}
    q = deque([(0, 0.0, 1), (1, 0.0, 0), (2, 0.0, 2), (3, 0.0, 3), (4, 0.0, 0)])
    taken, rej = serve.admit_requests(q, 0.0, caps, shapes)
    assert taken == [(1, 0), (4, 0)]
    assert [(r, s) for r, s, _ in rej] == [(0, 1), (2, 2), (3, 3)]
    assert all(isinstance(why, str) and why for _, _, why in rej)
    assert not q


class _Done:
    def query(self):
        return True


class _FakeSlot:
    """Stands in for a device slot: a launched batch finishes at once."""

    def __init__(self, fail_collect=False):
        self.done = _Done()
        self.requests = None
        self.resident_reqs = None
        self.fail_collect = fail_collect
        self.released = 0

    def collect(self, copy=False, pool=None):
        if self.fail_collect:
            raise torch.cuda.OutOfMemoryError("injected: out of device memory while growing edge buffers")
        out = {rid: {"status": "ok", "scene": si} for rid, si in self.requests[0]}
        out.update({rid: {"status": "ok", "scene": si, "resident": True} for rid, si in self.requests[1]})
        self.requests = None
        return out

    def request_ids(self):
        return [rid for rid, _ in self.requests[0]] + [rid for rid, _ in self.requests[1]]

    def release(self):
        self.released += 1
        self.requests = None


def _fake_server(shapes, caps, resident=None, fail_launch=(), fail_collect=False):
    srv = serve.Server.__new__(serve.Server)
    srv.caps = caps
    srv.shapes = shapes
    srv.pool = None
    srv.slots = [_FakeSlot(fail_collect), _FakeSlot(fail_collect)]
    srv._admit = lambda queue, now: serve.admit_requests(queue, now, caps, shapes, resident=resident or (lambda si: None))
    calls = []

    def launch(slot, reqs, res_reqs):
        calls.append((list(reqs), list(res_reqs)))
        if any(si in fail_launch for _, si in reqs):
            raise torch.cuda.OutOfMemoryError("injected: allocation failed at launch")
        slot.requests = (reqs, res_reqs)
    srv._launch = launch
    return srv, calls


def test_serve_loop_ends_with_rejected_requests():
    # the loop must end even when requests can never be admitted
    shapes = [(100, 20), (5000, 20)]
    srv, _ = _fake_server(shapes, {2: (1000, 16, 1000 * 32)})
    arrivals = np.linspace(0.0, 0.01, 20)
    scene = np.array([i % 2 for i in range(20)])
    lat, res, wall = srv.serve(arrivals, scene, keep_results=True)
    assert len(res) == 20
    for i in range(20):
        if scene[i] == 1:
            assert res[i]["status"] == "rejected" and "exceed" in res[i]["reason"]
        else:
            assert res[i]["status"] == "ok" and res[i]["scene"] == 0
    assert sorted(srv.rejected) == [i for i in range(20) if scene[i] == 1]
    assert np.all(lat >= 0)


def test_cancelled_requests_are_answered_once():
    # request 5 arrives late and is cancelled while queued; request 0 is
    # cancelled after it has been launched (its result is dropped)
    shapes = [(100, 20)]
    srv, _ = _fake_server(shapes, {2: (1000, 16, 1000 * 32)})
    arrivals = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.05])
    scene = np.zeros(6, dtype=int)
    lat, res, wall = srv.serve(arrivals, scene, keep_results=True, cancels=[(0.0, 0), (0.01, 5)])
    assert len(res) == 6
    assert res[5]["status"] == "cancelled" and res[0]["status"] == "cancelled"
    assert all(res[i]["status"] == "ok" for i in (1, 2, 3, 4))
    assert sorted(srv.cancelled) == [0, 5]


def test_failed_launch_and_collect_answer_error_and_go_on():
    # an allocation failure while launching a batch answers that batch's
    # requests with "error"; later batches still run
    shapes = [(100, 20), (100, 20)]
    caps = {2: (100, 16, 100 * 32)}  # one request per batch
    srv, calls = _fake_server(shapes, caps, fail_launch={1})
    arrivals = np.zeros(4)
    scene = np.array([0, 1, 0, 0])
    lat, res, wall = srv.serve(arrivals, scene, keep_results=True)
    assert res[1]["status"] == "error" and "allocation" in res[1]["reason"]
    assert [res[i]["status"] for i in (0, 2, 3)] == ["ok"] * 3
    assert srv.errors == [1] and sum(s.released for s in srv.slots) == 1
    # a failure while collecting answers every request of the batch
    srv, _ = _fake_server(shapes, caps, fail_collect=True)
    lat, res, wall = srv.serve(np.zeros(3), np.array([0, 1, 0]), keep_results=True)
    assert all(r["status"] == "error" and "collect" in r["reason"] for r in res.values())
    assert sorted(srv.errors) == [0, 1, 2]


def test_resident_requests_take_staging_not_class_capacity():
    # scene 0 is resident: its requests use no batch rows, only staging;
    # staging holds two of them per batch here
    shapes = [(400, 20), (400, 20)]
    caps = {2: (400, 16, 400 * 32)}
    need = {0: (400, 1000, 300, 501, 1)}
    stage = (800, 4000, 1000, 2000, 8)
    q = deque([(0, 0.0, 0), (1, 0.0, 1), (2, 0.0, 0), (3, 0.0, 0), (4, 0.0, 1)])
    taken, rej, res = serve.admit_requests(q, 0.0, caps, shapes, resident=need.get, stage=stage)
    assert taken == [(1, 1)] and res == [(0, 0), (2, 0)] and rej == []
    assert [r[0] for r in q] == [3, 4]
    taken, rej, res = serve.admit_requests(q, 0.0, caps, shapes, resident=need.get, stage=stage)
    assert taken == [(4, 1)] and res == [(3, 0)]
    # a resident scene whose results alone exceed the staging goes the batched way
    q = deque([(0, 0.0, 0)])
    taken, rej, res = serve.admit_requests(q, 0.0, caps, shapes, resident=need.get, stage=(100, 100, 100, 100, 8))
    assert taken == [(0, 0)] and res == []


def test_resident_pool_lru_budget_and_allocation_failure(monkeypatch):
    # footprints come from the library (cg_dict_size); entries in use are
    # never evicted; an allocation failure leaves the scene non-resident
    f = serve.resident_footprint(1000, 2000, 100)
    assert f > 4 * 1000 * 4 + 4 * 2000
    made = []

    class FakeScene:
        def __init__(self, si, ell, n_rows, ncells, nedges, device, alloc):
            alloc((1,), torch.int32, device)
            self.si, self.bytes, self.users = si, serve.resident_footprint(ncells, n_rows, ell), 0
            made.append(si)

        def build(self, sb, a, r0, stream):
            pass

    monkeypatch.setattr(serve, "ResidentScene", FakeScene)
    cpu_alloc = lambda shape, dtype, device: torch.empty(shape, dtype=dtype)
    pool = serve.ResidentPool(int(2.5 * f), device="cpu", alloc=cpu_alloc)
    for si in range(3):
        assert pool.add(si, 100, 2000, 1000, 10, None, 0, 0, None)
    assert list(pool.scenes) == [1, 2] and pool.evictions == 1   # scene 0 was the least recent
    pool.get(1).users = 1                                         # in flight: kept
    pool.get(1)
    assert pool.add(3, 100, 2000, 1000, 10, None, 0, 0, None)
    assert list(pool.scenes) == [1, 3] and pool.evictions == 2
    assert not pool.add(4, 100, 2000, 100000, 10, None, 0, 0, None)  # larger than the whole budget
    def oom(shape, dtype, device):
        raise torch.cuda.OutOfMemoryError("injected: out of device memory")
    pool2 = serve.ResidentPool(10 * f, device="cpu", alloc=oom)
    assert not pool2.add(0, 100, 2000, 1000, 10, None, 0, 0, None)
    assert pool2.alloc_failures == 1 and not pool2.scenes


def test_capacity_plan_fits_the_budget():
    # footprints come from the library's own workspace sizes; the plan picks
    # the largest power-of-two row capacity whose two slots fit the budget
    words = list(CLASS_WORDS)
    f1 = class_footprint(1 << 16, 256, (1 << 16) * 32, 8)
    f2 = class_footprint(1 << 17, 256, (1 << 17) * 32, 8)
    assert 1.8 < f2 / f1 < 2.2   # linear in the rows
    budget = 40 << 30
    rows, tot = serve.plan_capacity(words, budget, fraction=0.5)
    assert tot <= budget // 2
    bigger = 2 * sum(class_footprint(2 * rows, 4096, 2 * rows * 32 * (w - 1), w) for w in words)
    assert rows == 1 << 21 or bigger > budget // 2
