"""Admission logic of the serving loop, on the CPU (no device work)."""
from collections import deque

from paper_1503_06029_amd import serve
from paper_1503_06029_amd.batch import class_words


def test_class_words():
    assert [class_words(l) for l in (1, 32, 33, 96, 97, 224, 225, 480, 481, 992)] == [2, 2, 4, 4, 8, 8, 16, 16, 32, 32]


def test_admission_respects_arrival_and_capacity():
    shapes = [(100, 20), (300, 20), (50, 200), (400, 20)]
    caps = {2: (500, 8, 500 * 32), 8: (100, 2, 100 * 224)}
    q = deque([(0, 0.0, 0), (1, 0.1, 1), (2, 0.2, 2), (3, 0.3, 3), (4, 5.0, 0)])
    taken = serve.admit_requests(q, 1.0, caps, shapes)
    # request 3 (400 rows) does not fit after 0 and 1 (400 of 500 rows used); 4 has not arrived
    assert taken == [(0, 0), (1, 1), (2, 2)]
    assert [r[0] for r in q] == [3, 4]
    taken = serve.admit_requests(q, 1.0, caps, shapes)
    assert taken == [(3, 3)] and [r[0] for r in q] == [4]
    assert serve.admit_requests(q, 1.0, caps, shapes) == []
    assert serve.admit_requests(q, 6.0, caps, shapes) == [(4, 0)]


def test_admission_scene_limit_and_no_starvation():
    shapes = [(1, 10)]
    caps = {2: (1000, 3, 1000 * 32)}
    q = deque((i, 0.0, 0) for i in range(10))
    rounds = []
    while q:
        rounds.append([r for r, _ in serve.admit_requests(q, 0.0, caps, shapes)])
    assert rounds == [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9]]
