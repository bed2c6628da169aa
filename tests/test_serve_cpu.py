"""Batch formation of the serving loop (host logic, no device): the native
rule ``nurbs_server_admit`` through the C ABI."""
import pytest

pytest.importorskip("torch")

from paper_2104_14547_amd.serve import admit  # noqa: E402


def test_fifo_within_capacity():
    assert admit([0, 1, 2], [40, 40, 40], capacity=100, max_requests=10) == [0, 1]
    assert admit([2], [40], capacity=100, max_requests=10) == [0]


def test_head_of_line_request_is_not_overtaken():
    # request 1 does not fit after 0; the small request 2 behind it must wait too
    assert admit([0, 1, 2], [60, 60, 10], capacity=100, max_requests=10) == [0]
    assert admit([1, 2], [60, 10], capacity=100, max_requests=10) == [0, 1]


def test_same_surface_waits_for_next_batch_in_order():
    surfs = [7, 7, 3, 7, 5]
    assert admit(surfs, [10] * 5, capacity=1000, max_requests=10) == [0, 2, 4]
    # what stays queued, in arrival order: requests 1 and 3, both on surface 7
    assert admit([7, 7], [10, 10], capacity=1000, max_requests=10) == [0]


def test_max_requests_and_fixed_bytes():
    assert admit(list(range(10)), [1] * 10, capacity=1000, max_requests=4) == [0, 1, 2, 3]
    assert admit([0], [10], capacity=100, max_requests=100, fixed_bytes=95) == []
    assert admit([1], [5], capacity=100, max_requests=100, fixed_bytes=95) == [0]


def test_passed_over_requests_are_bounded():
    # 4 * max_requests repeats of a taken surface are passed over, no more
    surfs = [0] * 10 + [1]
    assert admit(surfs, [1] * 11, capacity=1000, max_requests=2) == [0]
    assert admit([0] * 8 + [1], [1] * 9, capacity=1000, max_requests=2) == [0, 8]


def test_empty_queue():
    assert admit([], [], capacity=10, max_requests=3) == []


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
