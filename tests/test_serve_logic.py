"""Admission logic and termination of the serving loop, on the CPU (no device work)."""
from collections import deque

import numpy as np

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

    def __init__(self):
        self.done = _Done()
        self.reqs = None

    def collect(self, copy=False):
        out = {rid: {"status": "ok", "scene": si} for rid, si in self.reqs}
        self.reqs = None
        return out


def test_serve_loop_ends_with_rejected_requests():
    # the loop must end even when requests can never be admitted
    srv = serve.Server.__new__(serve.Server)
    shapes = [(100, 20), (5000, 20)]
    srv.caps = {2: (1000, 16, 1000 * 32)}
    srv.slots = [_FakeSlot(), _FakeSlot()]
    srv._admit = lambda queue, now: serve.admit_requests(queue, now, srv.caps, shapes)

    def launch(slot, reqs):
        slot.reqs = reqs
    srv._launch = launch
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
