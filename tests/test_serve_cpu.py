"""Batch formation of the serving loop (host logic, no device)."""
import collections

import pytest

pytest.importorskip("torch")

from paper_2104_14547_amd.serve import Admission, Request  # noqa: E402


def req(rid, surf, nbytes):
    r = Request(surf, None, None, None)
    r.rid, r.nbytes = rid, nbytes
    return r


def ids(batch):
    return [r.rid for r in batch]


def test_fifo_within_capacity():
    q = collections.deque([req(0, 0, 40), req(1, 1, 40), req(2, 2, 40)])
    a = Admission(capacity=100, max_requests=10)
    assert ids(a.take(q)) == [0, 1]
    assert ids(q) == [2]
    assert ids(a.take(q)) == [2]
    assert not q


def test_head_of_line_request_is_not_overtaken():
    # request 1 does not fit after 0; the small request 2 behind it must wait too
    q = collections.deque([req(0, 0, 60), req(1, 1, 60), req(2, 2, 10)])
    a = Admission(capacity=100, max_requests=10)
    assert ids(a.take(q)) == [0]
    assert ids(q) == [1, 2]
    assert ids(a.take(q)) == [1, 2]


def test_same_surface_waits_for_next_batch_in_order():
    q = collections.deque([req(0, 7, 10), req(1, 7, 10), req(2, 3, 10), req(3, 7, 10), req(4, 5, 10)])
    a = Admission(capacity=1000, max_requests=10)
    assert ids(a.take(q)) == [0, 2, 4]
    assert ids(q) == [1, 3]          # kept, in arrival order
    assert ids(a.take(q)) == [1]
    assert ids(a.take(q)) == [3]


def test_max_requests_and_fixed_bytes():
    q = collections.deque([req(i, i, 1) for i in range(10)])
    a = Admission(capacity=1000, max_requests=4)
    assert ids(a.take(q)) == [0, 1, 2, 3]
    b = Admission(capacity=100, max_requests=100, fixed_bytes=95)
    r = req(0, 0, 10)
    assert not b.fits_alone(r)
    assert b.fits_alone(req(1, 1, 5))


def test_empty_queue():
    a = Admission(capacity=10, max_requests=3)
    assert a.take(collections.deque()) == []
