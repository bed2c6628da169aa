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


def test_knot_projection_orders_and_spaces():
    import numpy as np
    import torch
    from paper_2104_14547_amd.fit import project_knots
    rng = np.random.Generator(np.random.PCG64(0))
    for n in (1, 5, 60):
        gap = min(1e-3, 0.5 / (n + 1))
        ramp = torch.arange(1, n + 1, dtype=torch.float64) * gap
        for _ in range(20):
            x = torch.from_numpy(rng.uniform(-0.5, 1.5, n))
            y = x.clone()
            project_knots(y, ramp, 1.0 - (n + 1) * gap)
            full = torch.cat([torch.zeros(1, dtype=y.dtype), y, torch.ones(1, dtype=y.dtype)])
            assert torch.all(full[1:] - full[:-1] >= gap * (1 - 1e-9))
        # an already valid vector is left alone
        ok = torch.linspace(0, 1, n + 2, dtype=torch.float64)[1:-1]
        z = ok.clone()
        project_knots(z, ramp, 1.0 - (n + 1) * gap)
        assert torch.allclose(z, ok, rtol=0, atol=1e-12)
