"""Continuous-batching server of surface evaluation + gradient requests.

The surfaces (control nets, weights, knots) are uploaded once and stay
resident.  A request names a resident surface and brings its own parameter
grid (us, vs) and target points T; it gets back S on the grid and the
gradients of L = sum ||S - T||^2 with respect to the surface's control
points, weights and both knot vectors (the paper's forward and backward,
Sec. 3.1-3.2, per request).

Serving loop
------------
* Requests wait in a FIFO queue.  A batch is formed whenever an execution
  slot is free: requests are taken in arrival order while the batch's device
  bytes (parameters, points, dL/dS, targets, workspace, plan tables, packed
  outputs) fit the slot's memory; a request for a surface already in the
  forming batch waits for the next one (its gradient buffers would collide).
  A request larger than a whole slot is refused at submission.
* Each slot has its own stream, device arena and pinned host buffers.  The
  batch is packed on the host, copied up asynchronously, its plan is built
  into the slot's arena (nurbs_plan_create_in: no allocation, no
  synchronisation), and the forward, dL/dS = 2 (S - T), the backward, the
  gather of the requests' gradients and the copy back are queued on the
  slot's stream.  While one slot's batch runs, the next is formed from the
  requests that arrived meanwhile and launched on another slot, so batches
  overlap on the device.
* A batch's results are handed out when its stream has passed an event;
  latency is measured from a request's arrival to that moment.

Every result is the same alone and in any mix: a plan's tiles depend only on
each surface's own shape, and every reduction runs in a fixed order.
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
from .api import Context, NurbsError, _check, _ptr

_ALIGN = 256

# nurbs_desc as a numpy record type (six int32, then seven int64)
_DESC_DTYPE = np.dtype([(n, np.int32) for n in ("p", "q", "nu_c", "nv_c", "nu_s", "nv_s")] +
                       [(n, np.int64) for n in ("ctrl_off", "w_off", "ku_off", "kv_off", "us_off", "vs_off",
                                                "pts_off")], align=True)
assert _DESC_DTYPE.itemsize == ctypes.sizeof(N.nurbs_desc)


def _al(x: int) -> int:
    return (int(x) + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclass
class Request:
    surf: int
    us: np.ndarray
    vs: np.ndarray
    target: np.ndarray  # [nu_s, nv_s, 3]
    t_arrival: float = 0.0
    rid: int = 0
    # filled at submission
    nbytes: int = 0
    ws_bytes: int = 0
    table_bytes: int = 0
    future: Future = field(default_factory=Future)


@dataclass
class Result:
    pts: np.ndarray
    grad_ctrl: np.ndarray
    grad_w: np.ndarray
    grad_ku: np.ndarray
    grad_kv: np.ndarray
    latency: float = 0.0


class Admission:
    """Batch formation (host logic only, no device).

    ``take(pending)`` removes and returns the next batch from the deque
    ``pending``: arrival order, at most ``max_requests``, device bytes within
    ``capacity``, no surface twice.  It stops at the first request that does
    not fit (so a large request is not starved by small ones behind it)."""

    def __init__(self, capacity: int, max_requests: int, fixed_bytes: int = 0):
        self.capacity = int(capacity)
        self.max_requests = int(max_requests)
        self.fixed = int(fixed_bytes)

    def fits_alone(self, req: Request) -> bool:
        return self.fixed + req.nbytes <= self.capacity

    def take(self, pending: collections.deque) -> list:
        batch, used, surfs, skipped = [], self.fixed, set(), []
        while pending and len(batch) < self.max_requests:
            r = pending[0]
            if r.surf in surfs:
                skipped.append(pending.popleft())
                continue
            if used + r.nbytes > self.capacity:
                break
            pending.popleft()
            batch.append(r)
            used += r.nbytes
            surfs.add(r.surf)
        for r in reversed(skipped):
            pending.appendleft(r)
        return batch


class _Slot:
    """One batch in flight: its stream, device arena, pinned host mirror and
    the gradient buffers (pool-sized, one flat tensor)."""

    def __init__(self, dev, arena_bytes: int, grad_elems: int):
        self.stream = torch.cuda.Stream(device=dev)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
        self.host = torch.empty(arena_bytes, dtype=torch.uint8, pin_memory=True)
        self.gflat = torch.empty(grad_elems, dtype=torch.float32, device=dev)
        self.event = torch.cuda.Event()
        self.batch = None
        self.plan = None
        self.layout = None


class Server:
    """Serve eval+gradient requests on the surfaces of ``pool`` (a packed
    ``workloads.Batch``), kept resident on ``device``.

    slot_bytes   : device memory one in-flight batch may use (admission limit);
    n_slots      : batches in flight at once (each with its own stream);
    max_requests : requests per batch at most.
    """

    def __init__(self, pool, device: int = 0, slot_bytes: int = 1 << 30, n_slots: int = 3,
                 max_requests: int = 1024):
        self.dev = torch.device("cuda", device)
        self.ctx = Context(device)
        self.pool = pool
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        self.ctrl, self.w, self.ku, self.kv = (T(pool.ctrl), T(pool.w), T(pool.ku), T(pool.kv))
        self.shapes = np.asarray(pool.shapes, np.int64)
        self.offs = np.asarray(pool.offsets, np.int64)
        sizes = [pool.ctrl.size, pool.w.size, pool.ku.size, pool.kv.size]
        # the four gradient buffers are one flat tensor, so one gather packs a batch's outputs
        self.grad_base = np.cumsum([0] + sizes[:-1])
        self.slots = []
        for _ in range(n_slots):
            self.slots.append(_Slot(self.dev, slot_bytes, int(sum(sizes))))
        self.admission = Admission(slot_bytes, max_requests)
        self.pending = collections.deque()
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.running = False
        self.thread = None
        self.next_id = 0
        self.completed = []  # (rid, latency, points) for statistics
        self.batches = 0
        # per surface, once: the flat indices of its four gradient blocks in
        # the slot's gradient buffer (a batch's gather index is their
        # concatenation) and the counts of those blocks
        self._gidx, self._gcnt = [], []
        for surf in range(len(self.shapes)):
            cnts = self._grad_elems(surf)
            self._gcnt.append(cnts)
            self._gidx.append(np.concatenate([np.arange(int(self.grad_base[k] + self.offs[surf, k]),
                                                        int(self.grad_base[k] + self.offs[surf, k]) + c,
                                                        dtype=np.int64) for k, c in enumerate(cnts)]))
        self._size_cache = {}

    # -- request sizing -----------------------------------------------------
    def _desc(self, surf, nu_s, nv_s, us_off, vs_off, pts_off):
        d = N.nurbs_desc()
        p, q, nu_c, nv_c = (int(x) for x in self.shapes[surf, :4])
        d.p, d.q, d.nu_c, d.nv_c, d.nu_s, d.nv_s = p, q, nu_c, nv_c, int(nu_s), int(nv_s)
        o = self.offs[surf]
        d.ctrl_off, d.w_off, d.ku_off, d.kv_off = int(o[0]), int(o[1]), int(o[2]), int(o[3])
        d.us_off, d.vs_off, d.pts_off = int(us_off), int(vs_off), int(pts_off)
        return d

    def _grad_elems(self, surf):
        p, q, nu_c, nv_c = (int(x) for x in self.shapes[surf, :4])
        return nu_c * nv_c * 3, nu_c * nv_c, nu_c + p + 1, nv_c + q + 1

    def _size(self, req: Request):
        nu_s, nv_s = len(req.us), len(req.vs)
        key = (req.surf, nu_s, nv_s)
        hit = self._size_cache.get(key)
        if hit is None:
            # the plan's sizes depend on the shapes only: asked once per shape
            arr = (N.nurbs_desc * 1)(self._desc(req.surf, nu_s, nv_s, 0, 0, 0))
            tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
            _check(N.lib().nurbs_plan_create_in(self.ctx.handle, arr, 1, 0, None, 0, None, None, ctypes.byref(tb),
                                                ctypes.byref(wb)), self.ctx.handle)
            npts = nu_s * nv_s
            outs = sum(self._gcnt[req.surf])
            # us, vs, target, points, dL/dS, gradient index and packed outputs, workspace, tables
            nbytes = (_al(4 * (nu_s + nv_s)) + 3 * _al(12 * npts) + _al(8 * outs) + _al(4 * outs) +
                      _al(int(wb.value)) + int(tb.value))
            hit = self._size_cache[key] = (int(wb.value), int(tb.value), nbytes)
        req.ws_bytes, req.table_bytes, req.nbytes = hit

    # -- public API ---------------------------------------------------------
    def submit(self, surf: int, us, vs, target, t_arrival: float | None = None) -> Future:
        req = Request(int(surf), np.ascontiguousarray(us, np.float32), np.ascontiguousarray(vs, np.float32),
                      np.ascontiguousarray(target, np.float32).reshape(len(us), len(vs), 3))
        req.t_arrival = time.perf_counter() if t_arrival is None else t_arrival
        self._size(req)
        if not self.admission.fits_alone(req):
            req.future.set_exception(NurbsError(N.NURBS_EWORKSPACE, "request larger than a serving slot"))
            return req.future
        with self.lock:
            req.rid = self.next_id
            self.next_id += 1
            self.pending.append(req)
        self.wake.set()
        return req.future

    def start(self):
        if self.running:
            return self
        self.running = True
        self.thread = threading.Thread(target=self._loop, name="nurbs-serve", daemon=True)
        self.thread.start()
        return self

    def stop(self):
        self.running = False
        self.wake.set()
        if self.thread is not None:
            self.thread.join()
            self.thread = None
        for s in self.slots:
            if s.batch is not None:
                s.event.synchronize()
                self._finish(s)

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    # -- engine -------------------------------------------------------------
    def _loop(self):
        torch.cuda.set_device(self.dev)
        while self.running:
            progressed = False
            for s in self.slots:
                if s.batch is not None and s.event.query():
                    self._finish(s)
                    progressed = True
            for s in self.slots:
                if s.batch is None:
                    with self.lock:
                        batch = self.admission.take(self.pending)
                    if not batch:
                        break
                    try:
                        self._launch(s, batch)
                    except Exception as e:  # report to the callers, keep serving
                        for r in batch:
                            r.future.set_exception(e)
                        s.batch = None
                    progressed = True
            if not progressed:
                self.wake.wait(5e-5)
                self.wake.clear()

    def _launch(self, s: _Slot, batch: list):
        n = len(batch)
        # layout of the arena (bytes); the host staging buffer mirrors it
        lay = {}
        off = 0

        def region(name, nbytes):
            nonlocal off
            lay[name] = (off, int(nbytes))
            off += _al(nbytes)

        surfs = np.fromiter((r.surf for r in batch), np.int64, n)
        nus = np.fromiter((len(r.us) for r in batch), np.int64, n)
        nvs = np.fromiter((len(r.vs) for r in batch), np.int64, n)
        npts = nus * nvs
        n_uv, n_pts = int((nus + nvs).sum()), int(npts.sum())
        gsizes = [self._gcnt[sf] for sf in surfs]
        n_out = int(sum(sum(g) for g in gsizes))
        # one plan header for the batch, then every request's tile slots
        H = N.NURBS_PLAN_WS_HEADER
        ws_bytes = H + sum(r.ws_bytes - H for r in batch)
        region("uv", 4 * n_uv)
        region("target", 12 * n_pts)
        region("index", 8 * n_out)
        region("pts", 12 * n_pts)
        region("g", 12 * n_pts)
        region("out", 4 * n_out)
        region("ws", ws_bytes)
        region("tables", sum(r.table_bytes for r in batch))
        if off > s.arena.numel():
            raise NurbsError(N.NURBS_EWORKSPACE, "batch exceeds the slot arena")
        H = s.host.numpy()

        def hview(name, dtype):
            o, nb = lay[name]
            return H[o:o + nb].view(dtype)

        def dview(name, dtype):
            o, nb = lay[name]
            return s.arena[o:o + nb].view(dtype)

        # packing: one concatenation per array, straight into the pinned mirror
        np.concatenate([x for r in batch for x in (r.us, r.vs)], out=hview("uv", np.float32))
        np.concatenate([r.target.reshape(-1) for r in batch], out=hview("target", np.float32))
        np.concatenate([self._gidx[sf] for sf in surfs], out=hview("index", np.int64))
        # descriptors, filled column-wise in a record array laid out as nurbs_desc
        D = np.zeros(n, _DESC_DTYPE)
        sh = self.shapes[surfs]
        for k, name in enumerate(("p", "q", "nu_c", "nv_c")):
            D[name] = sh[:, k]
        D["nu_s"], D["nv_s"] = nus, nvs
        o = self.offs[surfs]
        for k, name in enumerate(("ctrl_off", "w_off", "ku_off", "kv_off")):
            D[name] = o[:, k]
        uv_start = np.concatenate([[0], np.cumsum(nus + nvs)[:-1]])
        D["us_off"], D["vs_off"] = uv_start, uv_start + nus
        D["pts_off"] = 3 * np.concatenate([[0], np.cumsum(npts)[:-1]])
        descs = D.ctypes.data_as(ctypes.POINTER(N.nurbs_desc))
        st = s.stream
        with torch.cuda.stream(st):
            up = lay["index"][0] + lay["index"][1]  # uv, target and index are contiguous at the front
            s.arena[:up].copy_(s.host[:up], non_blocking=True)
            tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
            plan = ctypes.c_void_p()
            o_t, n_t = lay["tables"]
            _check(N.lib().nurbs_plan_create_in(self.ctx.handle, descs, n, 0, _ptr(s.arena) + o_t, n_t,
                                                st.cuda_stream, ctypes.byref(plan), ctypes.byref(tb),
                                                ctypes.byref(wb)), self.ctx.handle)
            s.descs = D  # the plan copies the descriptors, but keep them until the batch is done
            s.plan = plan
            uv = dview("uv", torch.float32)
            pts, g = dview("pts", torch.float32), dview("g", torch.float32)
            ws_o, ws_n = lay["ws"]
            ws_ptr = _ptr(s.arena) + ws_o
            lib = N.lib()
            _check(lib.nurbs_plan_fwd(plan, _ptr(self.ctrl), _ptr(self.w), _ptr(self.ku), _ptr(self.kv), _ptr(uv),
                                      _ptr(uv), _ptr(pts), ws_ptr, ws_n, st.cuda_stream), self.ctx.handle)
            torch.sub(pts, dview("target", torch.float32), out=g)
            g.mul_(2.0)
            gf = s.gflat
            gptr = [_ptr(gf) + 4 * int(b) for b in self.grad_base]
            _check(lib.nurbs_plan_bwd(plan, _ptr(self.ctrl), _ptr(self.w), _ptr(self.ku), _ptr(self.kv), _ptr(uv),
                                      _ptr(uv), _ptr(g), gptr[0], gptr[1], gptr[2], gptr[3], N.NURBS_GRAD_ALL,
                                      ws_ptr, ws_n, st.cuda_stream), self.ctx.handle)
            out = dview("out", torch.float32)
            torch.index_select(gf, 0, dview("index", torch.int64), out=out)
            # results back: points and packed gradients
            for name in ("pts", "out"):
                o, nb = lay[name]
                s.host[o:o + nb].copy_(s.arena[o:o + nb], non_blocking=True)
            s.event.record(st)
        s.batch = batch
        s.layout = (lay, gsizes)
        self.batches += 1

    def _finish(self, s: _Slot):
        now = time.perf_counter()
        lay, gsizes = s.layout
        H = s.host.numpy()
        o, nb = lay["pts"]
        pts = H[o:o + nb].view(np.float32)
        o, nb = lay["out"]
        out = H[o:o + nb].view(np.float32)
        # one copy of each packed array out of the pinned mirror, then views
        pts = pts.copy()
        out = out.copy()
        cp = co = 0
        for r, gs in zip(s.batch, gsizes):
            nu_s, nv_s = len(r.us), len(r.vs)
            S = pts[3 * cp:3 * (cp + nu_s * nv_s)].reshape(nu_s, nv_s, 3)
            c0, c1, c2, c3 = gs
            p, q, nu_c, nv_c = (int(x) for x in self.shapes[r.surf, :4])
            res = Result(S, out[co:co + c0].reshape(nu_c, nv_c, 3), out[co + c0:co + c0 + c1].reshape(nu_c, nv_c),
                         out[co + c0 + c1:co + c0 + c1 + c2], out[co + c0 + c1 + c2:co + c0 + c1 + c2 + c3],
                         latency=now - r.t_arrival)
            co += c0 + c1 + c2 + c3
            self.completed.append((r.rid, res.latency, nu_s * nv_s))
            r.future.set_result(res)
            cp += nu_s * nv_s
        N.lib().nurbs_plan_destroy(s.plan)
        s.plan = None
        s.batch = None
        s.layout = None


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
    request's scheduled arrival to its result)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(requests)
    gaps = rng.exponential(1.0 / rate, n) if rate else np.zeros(n)
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
        for (s, us, vs, T), ta in zip(requests, arrivals):
            now = time.perf_counter()
            if ta > now:
                time.sleep(ta - now)
            futs.append(server.submit(s, us, vs, T, t_arrival=float(ta)))
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
