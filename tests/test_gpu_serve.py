"""Continuous-batching server on the GPU.

* a request's result is the same, bit for bit, alone (a batch of one) and in
  a mix of concurrent requests;
* results match the FP64 oracle at the point / gradient tolerances;
* memory admission: with small slots batches stay within the slot, and a
  request larger than a slot is refused;
* the per-request plain-launch baseline returns the same values.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2104_14547_amd import workloads as W  # noqa: E402
from paper_2104_14547_amd.api import NurbsError  # noqa: E402
from paper_2104_14547_amd.serve import PlainServer, Server, make_requests, run_load  # noqa: E402
from oracle import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def pool_small():
    return W.uneven_batch(3, n_surf=96, with_upstream=False)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in
               zip((a.pts, a.grad_ctrl, a.grad_w, a.grad_ku, a.grad_kv),
                   (b.pts, b.grad_ctrl, b.grad_w, b.grad_ku, b.grad_kv)))


def test_alone_equals_in_mix_and_oracle():
    pool = pool_small()
    reqs = make_requests(pool, 160, seed=11)
    with Server(pool, slot_bytes=256 << 20, n_slots=3, max_requests=64) as srv:
        _, mixed = run_load(srv, reqs, rate=None)
        assert srv.batches < len(reqs)  # requests were batched
    with Server(pool, slot_bytes=256 << 20, n_slots=1, max_requests=1) as one:
        _, alone = run_load(one, reqs[:40], rate=None)
    for k in range(40):
        assert same(mixed[k], alone[k]), f"request {k}: result differs alone vs in the mix"
    # a few against the oracle
    for k in range(0, 160, 23):
        s, us, vs, T = reqs[k]
        d = pool.surface(s)
        S = O.surface_fwd(d["ctrl"], d["w"], d["ku"], d["kv"], d["p"], d["q"], us, vs, local=True)
        g = 2.0 * (mixed[k].pts.astype(np.float32) - T)  # the server's own dL/dS, as the kernels saw it
        gc, gw, gu, gv = O.surface_bwd(d["ctrl"], d["w"], d["ku"], d["kv"], d["p"], d["q"], us, vs,
                                       g.astype(np.float32).astype(np.float64), local=True)
        diag = np.linalg.norm(S.reshape(-1, 3).max(0) - S.reshape(-1, 3).min(0))
        assert np.linalg.norm((mixed[k].pts - S).reshape(-1, 3), axis=1).max() <= 1e-5 * diag
        for got, want in ((mixed[k].grad_ctrl, gc), (mixed[k].grad_w, gw), (mixed[k].grad_ku, gu),
                          (mixed[k].grad_kv, gv)):
            assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max()


def test_memory_admission_small_slots():
    pool = pool_small()
    reqs = make_requests(pool, 40, seed=12)
    with Server(pool, slot_bytes=8 << 20, n_slots=2, max_requests=64) as srv:
        sizes = []
        for s, us, vs, T in reqs:
            f = srv.submit(s, us, vs, T)
            sizes.append(f)
        res = [f.result() for f in sizes]
        assert len(res) == 40
        assert srv.batches > 1
    # a request that cannot fit any slot is refused, the server keeps going
    big = W.uneven_batch(3, n_surf=1, with_upstream=False)
    d = big.surface(0)
    with Server(big, slot_bytes=1 << 20, n_slots=1) as srv:
        us = np.linspace(0, 1, 256, dtype=np.float32)
        f = srv.submit(0, us, us, np.zeros((256, 256, 3), np.float32))
        with pytest.raises(NurbsError):
            f.result()
        f2 = srv.submit(0, d["us"][:4], d["vs"][:4], np.zeros((4, 4, 3), np.float32))
        assert f2.result().pts.shape == (4, 4, 3)


def test_plain_baseline_matches_server():
    pool = pool_small()
    reqs = make_requests(pool, 12, seed=13)
    with Server(pool, slot_bytes=64 << 20) as srv:
        _, a = run_load(srv, reqs, rate=None)
    with PlainServer(pool) as plain:
        _, b = run_load(plain, reqs, rate=None)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x.pts, y.pts, rtol=0, atol=1e-5)
        for u, v in zip((x.grad_ctrl, x.grad_w, x.grad_ku, x.grad_kv), (y.grad_ctrl, y.grad_w, y.grad_ku, y.grad_kv)):
            np.testing.assert_allclose(u, v, rtol=0, atol=1e-4 * max(np.abs(v).max(), 1e-30))


def test_concurrent_submitters_and_caller_buffers():
    # four client threads submit at once, two of them into their own output
    # buffers; every result is bitwise the one of the same request served alone
    import threading
    pool = pool_small()
    reqs = make_requests(pool, 120, seed=14)
    with Server(pool, slot_bytes=128 << 20, n_slots=1, max_requests=1) as one:
        _, alone = run_load(one, reqs, rate=None)
    got = [None] * len(reqs)
    with Server(pool, slot_bytes=128 << 20, n_slots=3, max_requests=32) as srv:
        def client(t):
            mine = range(t, len(reqs), 4)
            futs = []
            for k in mine:
                s, us, vs, T = reqs[k]
                out = np.full(srv.out_floats(s, len(us), len(vs)), np.nan, np.float32) if t % 2 else None
                futs.append((k, srv.submit(s, us, vs, T, out=out)))
            for k, f in futs:
                got[k] = f.result()
        th = [threading.Thread(target=client, args=(t,)) for t in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for k in range(len(reqs)):
        assert same(got[k], alone[k]), f"request {k}: differs from the request served alone"


def test_large_request_spans_many_segment_pieces():
    # 200 x 180 samples: the residual and the copies run in several pieces of
    # at most 16384 floats; the result matches the per-request baseline
    pool = pool_small()
    us = np.linspace(0.0, 1.0, 200, dtype=np.float32)
    vs = np.linspace(0.0, 1.0, 180, dtype=np.float32)
    rng = np.random.Generator(np.random.PCG64(15))
    T = rng.uniform(-0.2, 0.2, (200, 180, 3)).astype(np.float32)
    reqs = [(5, us, vs, T), (6, us[:37], vs[:41], T[:37, :41].copy())]
    with Server(pool, slot_bytes=64 << 20) as srv:
        _, a = run_load(srv, reqs, rate=None)
    with PlainServer(pool) as plain:
        _, b = run_load(plain, reqs, rate=None)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x.pts, y.pts, rtol=0, atol=1e-5)
        for u, v in zip((x.grad_ctrl, x.grad_w, x.grad_ku, x.grad_kv), (y.grad_ctrl, y.grad_w, y.grad_ku, y.grad_kv)):
            np.testing.assert_allclose(u, v, rtol=0, atol=1e-4 * max(np.abs(v).max(), 1e-30))
