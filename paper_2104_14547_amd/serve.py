"""Continuous-batching server of surface evaluation + gradient requests.

The surfaces (control nets, weights, knots) are uploaded once and stay
resident.  A request names a resident surface and brings its own parameter
grid (us, vs) and target points T; it gets back S on the grid and the
gradients of L = sum ||S - T||^2 with respect to the surface's control
points, weights and both knot vectors (the paper's forward and backward,
Sec. 3.1-3.2, per request).

``Server`` is a handle on the native server (``nurbs_server_*`` in the C
ABI), which runs the serving loop in two threads of its own:

* Requests wait in a FIFO queue.  A batch is formed whenever an execution
  slot is free: requests are taken in arrival order while the batch's device
  bytes (parameters, targets, points, dL/dS, packed outputs, workspace, plan
  tables) fit the slot's memory; a request for a surface already in the
  forming batch waits for the next one (its gradient buffers would collide).
  A request larger than a whole slot is refused at submission.
* Each slot has its own stream, device arena and pinned host buffer.  The
  engine thread packs the batch into the pinned buffer and queues on the
  slot's stream the copy up, the plan's tables (nurbs_plan_create_in: no
  allocation, no synchronisation), the forward, dL/dS = 2 (S - T), the
  backward, the gather of each request's gradients next to its points and
  the copy back.  While one slot's batch runs, the next is formed from the
  requests that arrived meanwhile and launched on another slot.
* The completion thread waits for each slot's event, copies every request's
  block into the caller's output array and wakes its waiters; latency is
  measured from a request's arrival to that moment.

Python only submits (one call per request) and waits.  Every result is the
same alone and in any mix: a plan's tiles depend only on each surface's own
shape, and every reduction runs in a fixed order.

``PlainServer`` is the per-request baseline: one request at a time through
the uniform-batch calls.
"""
from __future__ import annotations

import collections
import ctypes
import gc
import sys
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as N
from .api import NurbsError, _check, _ptr


@dataclass
class Request:
    surf: int
    us: np.ndarray
    vs: np.ndarray
    target: np.ndarray  # [nu_s, nv_s, 3]
    t_arrival: float = 0.0
    rid: int = 0
    future: Future = field(default_factory=Future)


@dataclass
class Result:
    pts: np.ndarray
    grad_ctrl: np.ndarray
    grad_w: np.ndarray
    grad_ku: np.ndarray
    grad_kv: np.ndarray
    latency: float = 0.0


def admit(surfs, nbytes, capacity: int, max_requests: int, fixed_bytes: int = 0) -> list:
    """The server's batch-formation rule on a queue given as parallel lists
    (surface, device bytes) in arrival order: the indices of the requests the
    next batch takes (host logic, ``nurbs_server_admit``)."""
    n = len(surfs)
    sf = (ctypes.c_int32 * max(n, 1))(*surfs)
    nb = (ctypes.c_size_t * max(n, 1))(*nbytes)
    take = (ctypes.c_int32 * max(n, 1))()
    k = ctypes.c_int()
    _check(N.lib().nurbs_server_admit(sf, nb, n, int(capacity), int(fixed_bytes), int(max_requests), take,
                                      ctypes.byref(k)))
    return list(take[:k.value])


class PackedResult:
    """A served request's outputs: views of the one array the native server
    wrote (points, then the four gradients), made when first read."""

    __slots__ = ("_o", "_nu", "_nv", "_geo", "latency")

    def __init__(self, out, nu, nv, geo, latency):
        self._o, self._nu, self._nv, self._geo, self.latency = out, nu, nv, geo, latency

    @property
    def pts(self):
        return self._o[:3 * self._nu * self._nv].reshape(self._nu, self._nv, 3)

    def _grad(self, k):
        nu_c, nv_c, *cnt = self._geo
        a = 3 * self._nu * self._nv + sum(cnt[:k])
        return self._o[a:a + cnt[k]]

    @property
    def grad_ctrl(self):
        return self._grad(0).reshape(self._geo[0], self._geo[1], 3)

    @property
    def grad_w(self):
        return self._grad(1).reshape(self._geo[0], self._geo[1])

    @property
    def grad_ku(self):
        return self._grad(2)

    @property
    def grad_kv(self):
        return self._grad(3)


class Pending:
    """A submitted request.  ``result()`` blocks until it has been served and
    returns a ``PackedResult``, or raises ``NurbsError``."""

    __slots__ = ("_srv", "id", "_keep", "_out", "_geo", "_nu", "_nv", "_res", "_err")

    def __init__(self, srv, rid, keep, out, geo, nu, nv, err=None):
        self._srv, self.id, self._keep, self._out, self._geo = srv, rid, keep, out, geo
        self._nu, self._nv, self._res, self._err = nu, nv, None, err

    def done(self) -> bool:
        return self._res is not None or self._err is not None or self._srv._finished_below() > self.id

    def result(self):
        if self._res is None and self._err is None:
            if self._srv._hv is None:
                raise NurbsError(N.NURBS_EINVAL, "the server was stopped before this request was resolved")
            rc, lat = self._srv._fast.wait(self._srv._hv, self.id)
            if rc != N.NURBS_OK:
                self._err = NurbsError(rc, N.lib().nurbs_server_last_error(self._srv._h).decode())
            else:
                self._res = PackedResult(self._out, self._nu, self._nv, self._geo, lat)
            self._keep = None
        if self._err is not None:
            raise self._err
        return self._res


class Server:
    """Serve eval+gradient requests on the surfaces of ``pool`` (a packed
    ``workloads.Batch``), kept resident on ``device``: a thin handle on the
    native server (``nurbs_server_*``), whose engine and completion threads
    form the batches, launch them and copy the results out.

    slot_bytes   : device memory one in-flight batch may use (admission limit);
    n_slots      : batches in flight at once (each with its own stream);
    max_requests : requests per batch at most.
    """

    def __init__(self, pool, device: int = 0, slot_bytes: int = 1 << 30, n_slots: int = 3,
                 max_requests: int = 1024):
        self.dev = torch.device("cuda", device)
        self.pool = pool
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        self.ctrl, self.w, self.ku, self.kv = (T(pool.ctrl), T(pool.w), T(pool.ku), T(pool.kv))
        torch.cuda.synchronize(self.dev)
        shapes = np.asarray(pool.shapes, np.int64)
        offs = np.asarray(pool.offsets, np.int64)
        n = len(shapes)
        D = (N.nurbs_desc * n)()
        self._geo = []
        for k in range(n):
            p, q, nu_c, nv_c = (int(x) for x in shapes[k, :4])
            d = D[k]
            d.p, d.q, d.nu_c, d.nv_c = p, q, nu_c, nv_c
            d.ctrl_off, d.w_off, d.ku_off, d.kv_off = (int(x) for x in offs[k, :4])
            self._geo.append((nu_c, nv_c, 3 * nu_c * nv_c, nu_c * nv_c, nu_c + p + 1, nv_c + q + 1))
        # floats of gradients per surface, after the 3 nu_s nv_s of points
        self._gout = [sum(g[2:]) for g in self._geo]
        h = ctypes.c_void_p()
        L = N.lib()
        _check(L.nurbs_server_create(int(device), D, n, _ptr(self.ctrl), _ptr(self.w), _ptr(self.ku),
                                     _ptr(self.kv), int(n_slots), int(slot_bytes), int(max_requests),
                                     ctypes.byref(h)))
        self._h = h
        self._hv = h.value
        self._fast = N.serve_py()
        self._live = collections.deque()  # requests whose buffers the native side may still use
        self._since_prune = 0
        self._lock = threading.Lock()

    def _finished_below(self) -> int:
        f = ctypes.c_int64()
        N.lib().nurbs_server_stats(self._h, None, None, ctypes.byref(f))
        return f.value

    @property
    def batches(self) -> int:
        b = ctypes.c_int64()
        N.lib().nurbs_server_stats(self._h, ctypes.byref(b), None, None)
        return b.value

    def busy(self):
        """Host seconds the engine and completion threads spent on batches."""
        e, c = ctypes.c_double(), ctypes.c_double()
        N.lib().nurbs_server_busy(self._h, ctypes.byref(e), ctypes.byref(c))
        return e.value, c.value

    def out_floats(self, surf: int, nu_s: int, nv_s: int) -> int:
        """Floats of a request's output array: 3 nu_s nv_s points, then the
        four gradients."""
        return 3 * int(nu_s) * int(nv_s) + self._gout[int(surf)]

    def submit(self, surf: int, us, vs, target, t_arrival: float | None = None, out=None) -> Pending:
        """Queue a request; thread-safe.  Returns at once with a ``Pending``.

        out : optional float32 C-contiguous array of at least
              ``out_floats(surf, nu_s, nv_s)`` floats that receives the results
              (a client that reuses its buffers); default: a new array."""
        us = np.ascontiguousarray(us, np.float32)
        vs = np.ascontiguousarray(vs, np.float32)
        target = np.ascontiguousarray(target, np.float32)
        nu, nv = us.shape[0], vs.shape[0]
        if target.size != 3 * nu * nv:
            raise ValueError("target must hold nu_s * nv_s * 3 floats")
        surf = int(surf)
        need = 3 * nu * nv + self._gout[surf]
        if out is None:
            out = np.empty(need, np.float32)
        elif out.dtype != np.float32 or out.size < need or not out.flags.c_contiguous:
            raise ValueError(f"out must be a contiguous float32 array of at least {need} floats")
        rc, rid = self._fast.submit(self._hv, surf, us, vs, target, out, -1.0 if t_arrival is None else t_arrival)
        if rc == N.NURBS_EWORKSPACE:
            return Pending(self, -1, None, None, None, nu, nv,
                           err=NurbsError(rc, "request larger than a serving slot"))
        if rc != N.NURBS_OK:
            raise NurbsError(rc, "submit")
        f = Pending(self, rid, (us, vs, target), out, self._geo[surf], nu, nv)
        with self._lock:
            self._live.append(f)
            self._since_prune += 1
            if self._since_prune >= 256:
                # resolve the finished requests (their results and latencies
                # are read now, without waiting) and let go of their buffers
                self._since_prune = 0
                below = self._finished_below()
                live = self._live
                while live and live[0].id < below:
                    try:
                        live.popleft().result()
                    except NurbsError:
                        pass
        return f

    def start(self):
        return self

    def stop(self):
        """Serves what is queued and resolves every request, then stops the
        native threads and frees the slots."""
        if self._h:
            with self._lock:
                for f in self._live:
                    try:
                        f.result()
                    except NurbsError:
                        pass
                self._live.clear()
            N.lib().nurbs_server_destroy(self._h)
            self._h = None
            self._hv = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


class PlainServer:
    """Baseline: one request at a time, first come first served, each with
    its own plain uniform-batch launches (B = 1) and a synchronous copy back.
    Same interface as ``Server``."""

    def __init__(self, pool, device: int = 0):
        from .api import surface_bwd, surface_fwd
        self._fwd, self._bwd = surface_fwd, surface_bwd
        self.dev = torch.device("cuda", device)
        self.pool = pool
        self.surf = {}
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        for s in range(pool.n):
            d = pool.surface(s)
            self.surf[s] = (T(d["ctrl"]), T(d["w"]), T(d["ku"]), T(d["kv"]), d["p"], d["q"])
        self.pending = collections.deque()
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.running = False
        self.thread = None
        self.completed = []
        self.next_id = 0

    def submit(self, surf: int, us, vs, target, t_arrival: float | None = None) -> Future:
        req = Request(int(surf), np.ascontiguousarray(us, np.float32), np.ascontiguousarray(vs, np.float32),
                      np.ascontiguousarray(target, np.float32).reshape(len(us), len(vs), 3))
        req.t_arrival = time.perf_counter() if t_arrival is None else t_arrival
        with self.lock:
            req.rid = self.next_id
            self.next_id += 1
            self.pending.append(req)
        self.wake.set()
        return req.future

    def start(self):
        self.running = True
        self.thread = threading.Thread(target=self._loop, name="nurbs-plain", daemon=True)
        self.thread.start()
        return self

    def stop(self):
        self.running = False
        self.wake.set()
        if self.thread is not None:
            self.thread.join()
            self.thread = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    def _loop(self):
        torch.cuda.set_device(self.dev)
        while self.running or self.pending:
            with self.lock:
                r = self.pending.popleft() if self.pending else None
            if r is None:
                if not self.running:
                    break
                self.wake.wait(5e-5)
                self.wake.clear()
                continue
            ctrl, w, ku, kv, p, q = self.surf[r.surf]
            us = torch.from_numpy(r.us).to(self.dev, non_blocking=False)
            vs = torch.from_numpy(r.vs).to(self.dev, non_blocking=False)
            tg = torch.from_numpy(r.target).to(self.dev, non_blocking=False)
            S = self._fwd(ctrl, w, ku, kv, p, q, us, vs)
            g = (S - tg) * 2.0
            gc, gw, gu, gv = self._bwd(ctrl, w, ku, kv, p, q, us, vs, g)
            res = Result(S.cpu().numpy(), gc.cpu().numpy(), gw.cpu().numpy(), gu.cpu().numpy(), gv.cpu().numpy())
            res.latency = time.perf_counter() - r.t_arrival
            self.completed.append((r.rid, res.latency, len(r.us) * len(r.vs)))
            r.future.set_result(res)


def make_requests(pool, n: int, seed: int = 4):
    """n requests drawn uniformly from the pool's surfaces, each on that
    surface's own parameter grid, with targets (u, v, z), z ~ U(-0.2, 0.2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        s = int(rng.integers(0, pool.n))
        d = pool.surface(s)
        us, vs = d["us"], d["vs"]
        T = np.empty((len(us), len(vs), 3), np.float32)
        T[..., 0] = us[:, None]
        T[..., 1] = vs[None, :]
        T[..., 2] = rng.uniform(-0.2, 0.2, (len(us), len(vs))).astype(np.float32)
        out.append((s, us, vs, T))
    return out


def run_load(server, requests, rate: float | None, seed: int = 5):
    """Submit ``requests`` to a started server, as a Poisson stream of
    ``rate`` requests/s (None: all at once, closed loop), and wait for every
    result.  Returns throughput and latency statistics (latency from each
    request's scheduled arrival to its result).

    For a server that takes output buffers, the client allocates and touches
    them before the clock starts, as a client that reuses its buffers would
    have them: first-touch page faults of fresh host memory are the
    client's allocation cost, not the server's."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(requests)
    gaps = rng.exponential(1.0 / rate, n) if rate else np.zeros(n)
    outs = [None] * n
    if hasattr(server, "out_floats"):
        sizes = [server.out_floats(s, len(us), len(vs)) for (s, us, vs, _) in requests]
        buf = np.empty(sum(sizes), np.float32)
        buf.fill(0.0)
        ends = np.cumsum(sizes)
        outs = [buf[e - k:e] for e, k in zip(ends, sizes)]
    # no cyclic garbage collection while the clock runs: its pauses (tens of
    # ms) would show up as latency of whichever requests were in flight
    gc.collect()
    gc_was_on = gc.isenabled()
    gc.disable()
    # the client (this thread) and the serving thread share the interpreter
    # lock; at the default 5 ms switch interval a busy client can hold the
    # server off for whole milliseconds, which shows up as tail latency
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    try:
        t0 = time.perf_counter()
        arrivals = t0 + np.cumsum(gaps)
        futs = []
        for (s, us, vs, T), ta, o in zip(requests, arrivals, outs):
            # wait for the scheduled arrival: sleep only through long gaps
            # (the OS wakes a sleeper tens of microseconds late, and requests
            # would then go out in bursts behind their schedule), spin on the
            # clock for the rest
            now = time.perf_counter()
            if ta - now > 2e-3:
                time.sleep(ta - now - 1e-3)
            while time.perf_counter() < ta:
                pass
            if o is None:
                futs.append(server.submit(s, us, vs, T, t_arrival=float(ta)))
            else:
                futs.append(server.submit(s, us, vs, T, t_arrival=float(ta), out=o))
        results = [f.result() for f in futs]
        t1 = time.perf_counter()
    finally:
        sys.setswitchinterval(switch)
        if gc_was_on:
            gc.enable()
    lat = np.array([r.latency for r in results])
    pts = sum(len(r[1]) * len(r[2]) for r in requests)
    return {"requests": n, "rate_offered": rate, "seconds": t1 - t0, "req_per_s": n / (t1 - t0),
            "pts_per_s": pts / (t1 - t0), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3)}, results
