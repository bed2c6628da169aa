#!/usr/bin/env python
"""Throughput of batched NURBS surface evaluation + adjoint on one MI355X.

Workload (default): the uneven batch -- 4096 surfaces, degrees p, q in 1..5,
control sides 4..48 and sample sides 16..256 (log-uniform), non-uniform
clamped knots with 10% repeated interior knots -- run as one ragged plan:
one persistent forward launch, one persistent backward launch, its
persistent gather (the v-contraction of the tile accumulators on the matrix
cores) and the per-surface finalize.  A step is forward + backward (all four gradients)
over the whole batch with every input resident in HBM; the upstream
gradient dL/dS is a fixed synthetic array (see workloads.uneven_batch).

Prints ONE JSON line: metric, value (surface points per second of
forward + backward), roofline of the dominant kernel (algorithmic bytes per
launch / its average duration, from HIP events recorded around each kernel
during the timed steps), the FP64 oracle's throughput on a bounded sample of
the same batch (cpu_baseline) and the parity errors of the timed outputs on
every surface.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FLUSH_BYTES = 512 << 20  # larger than the 256 MB MALL
METRIC = "surface pts/s fwd+bwd (fp32, err≤1e-5 vs fp64 oracle); p50/p99 served latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# host code of the serving engine: no part of the kernels or of their launches
SERVING_SOURCES = ("serve_py.c", "server.hip")


def kernel_source_digest() -> str:
    """Digest of the sources the kernels and their launches are built from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2104_14547_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in SERVING_SOURCES:
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(shapes):
    """Bytes the method must move, per kernel (float32).

    forward : write S (12 B/pt), read P and W (16 B/control point), read the
              samples (4 B each) and knots (4 B each);
    backward: read dL/dS (12 B/pt), read P and W, samples and knots;
    gather  : none (it reads and writes the backward's workspace only);
    finalize: write dL/dP and dL/dW (16 B/control point), dL/dU, dL/dV (4 B/knot).
    Total 24 B/pt + 48 B/cp + 8 B/sample + 12 B/knot."""
    import numpy as np
    s = np.asarray(shapes, np.int64)
    pts = int((s[:, 4] * s[:, 5]).sum())
    cps = int((s[:, 2] * s[:, 3]).sum())
    smp = int((s[:, 4] + s[:, 5]).sum())
    kn = int((s[:, 2] + s[:, 0] + 1 + s[:, 3] + s[:, 1] + 1).sum())
    return {"points": pts, "control_points": cps, "samples": smp, "knots": kn,
            "fwd": 12 * pts + 16 * cps + 4 * smp + 4 * kn,
            "bwd": 12 * pts + 16 * cps + 4 * smp + 4 * kn,
            "gat": 0,
            "fin": 16 * cps + 4 * kn}


def traffic_for(kernel: str, workload: str, chosen: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources with the same schedule and the
    same tile size for this kernel's direction; else None."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    tile = chosen["fwd_tile_points"] if kernel == "k_fwd_plan" else chosen["bwd_tile_points"]
    for r in rec.get("records", []):
        if r["kernel"] == kernel and r["tile_points"] == tile and r["schedule"] == chosen.get("schedule"):
            return r["hbm_bytes_per_launch"]
    return None


def make_flush(torch, dev):
    """Two FLUSH_BYTES halves for evict_mall: one written, one read."""
    f = torch.empty(2 * FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
    f.fill_(0.0)
    return f


def evict_mall(torch, flush):
    """Evict the caches before a timed step: a FLUSH_BYTES scratch write (the
    first half of ``flush``, larger than the 256 MB MALL), then a read of the
    second half, and a wait for both.  The read replaces the write's dirty
    lines with clean ones, so the step starts with the caches holding none of
    its inputs and does not pay for writing the scratch data back to HBM
    (measured: a write-only flush added about 40 us to the uneven-batch step,
    most of it in the first kernel)."""
    half = flush.numel() // 2
    flush[:half].fill_(0.0)
    torch.sum(flush[half:])
    torch.cuda.synchronize()


def timed_steps(torch, step, n: int, flush=None):
    """Run ``step`` n times between HIP events on the current stream; with
    ``flush`` (a large device buffer), evict the MALL before each step,
    outside the events.  Returns the per-step times in ms."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        if flush is not None:
            evict_mall(torch, flush)
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def cpu_baseline(batch, sample: int, seed: int = 17):
    import numpy as np
    from oracle import oracle as O
    g = np.random.Generator(np.random.PCG64(seed))
    idx = sorted(g.choice(batch.n, min(sample, batch.n), replace=False).tolist())
    sub = batch.subset(idx)
    threads = O.max_threads()
    t0 = time.perf_counter()
    O.fwd(sub, local=True)
    O.bwd(sub, sub.upstream.astype(np.float64), local=True)
    dt = time.perf_counter() - t0
    return {"value": sub.n_points / dt, "unit": "pts/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} of {batch.n} surfaces ({sub.n_points} points), FP64 oracle in "
                      f"local (non-zero span) mode, forward + backward, {dt:.2f} s on {threads} threads"}


def per_surface_errors(batch, pts, grads, S, G):
    """Per-surface parity errors of GPU outputs against oracle outputs S, G
    (packed layouts): the point error relative to the bounding-box diagonal
    of the oracle's points, and each gradient's max error relative to its
    largest oracle magnitude."""
    sh = np.asarray(batch.shapes, np.int64)
    off = np.asarray(batch.offsets, np.int64)
    npts = sh[:, 4] * sh[:, 5]
    live = npts > 0
    got = pts[: batch.n_pts_floats].astype(np.float64).reshape(-1, 3)
    want = S.reshape(-1, 3)
    # surfaces are packed back to back, so reduceat over their first points
    starts = (off[:, 6] // 3)[live]
    err = np.linalg.norm(got - want, axis=1)
    perr = np.maximum.reduceat(err, starts)
    diag = np.linalg.norm(np.maximum.reduceat(want, starts, axis=0) - np.minimum.reduceat(want, starts, axis=0),
                          axis=1)
    point_rel = perr / np.where(diag > 0, diag, 1.0)
    sizes = (sh[:, 2] * sh[:, 3] * 3, sh[:, 2] * sh[:, 3], sh[:, 2] + sh[:, 0] + 1, sh[:, 3] + sh[:, 1] + 1)
    grad_rel = []
    for k in range(4):
        a = grads[k].astype(np.float64)
        b = G[k]
        st = off[:, k]
        d = np.maximum.reduceat(np.abs(a - b), st)
        m = np.maximum.reduceat(np.abs(b), st)
        grad_rel.append(np.where(m > 0, d / np.where(m > 0, m, 1.0), d))
        assert (np.diff(st) == sizes[k][:-1]).all()
    return point_rel, np.max(np.stack(grad_rel), axis=0)


def parity_all(batch, pts, grads, pts_tol=1e-5, grad_tol=1e-4):
    """Parity of the timed outputs on every surface of the batch."""
    from oracle import oracle as O
    S = O.fwd(batch, local=True)
    G = O.bwd(batch, batch.upstream.astype(np.float64), local=True)
    point_rel, grad_rel = per_surface_errors(batch, pts, grads, S, G)
    ok = bool((point_rel <= pts_tol).all() and (grad_rel <= grad_tol).all())
    return {"surfaces": batch.n, "max_point_err_rel_bbox": float(point_rel.max()),
            "max_grad_err_rel_inf": float(grad_rel.max()), "pass": ok}


def served_leg(batch, n_req: int, seed: int = 4):
    """Continuous-batching server on the batch's surfaces (resident): closed-
    loop saturation, then Poisson arrivals at 0.5x, 0.8x and 1.0x of it (each
    after an untimed run as long at the same rate), and the per-request
    plain-launch baseline at the same rates (fewer requests: it saturates far
    earlier)."""
    from paper_2104_14547_amd.serve import PlainServer, Server, make_requests, run_load
    reqs = make_requests(batch, n_req, seed=seed)
    out = {"requests_per_rate": n_req, "rates": [],
           "note": "native engine; the client's output arrays are allocated and touched before each run's clock "
                   "starts; latency from each request's scheduled arrival to its result"}
    with Server(batch, slot_bytes=1 << 30, n_slots=3, max_requests=512) as srv:
        run_load(srv, reqs[: min(200, n_req)], rate=None)  # warm-up
        b0, (e0, c0) = srv.batches, srv.busy()
        sat, _ = run_load(srv, reqs, rate=None)
        b1, (e1, c1) = srv.batches, srv.busy()
        out["saturation_req_s"] = sat["req_per_s"]
        out["saturation_pts_s"] = sat["pts_per_s"]
        # host time of the native threads at saturation, per request
        out["saturation_requests_per_batch"] = n_req / max(1, b1 - b0)
        out["engine_us_per_request"] = (e1 - e0) / n_req * 1e6
        out["completion_us_per_request"] = (c1 - c0) / n_req * 1e6
        for f in (0.5, 0.8, 1.0):
            # an untimed run of the same length at the same rate first: the
            # measured run starts in steady state
            run_load(srv, reqs, rate=f * sat["req_per_s"], seed=seed + 2)
            st, _ = run_load(srv, reqs, rate=f * sat["req_per_s"], seed=seed + 1)
            st["load"] = f
            out["rates"].append(st)
        out["batches"] = srv.batches
    n_plain = min(n_req, 2000)
    plain = {"requests_per_rate": n_plain, "rates": []}
    with PlainServer(batch) as ps:
        run_load(ps, reqs[:20], rate=None)
        st, _ = run_load(ps, reqs[:n_plain], rate=None)
        plain["saturation_req_s"] = st["req_per_s"]
        for f in (0.5, 0.8, 1.0):
            st, _ = run_load(ps, reqs[:n_plain], rate=f * out["saturation_req_s"], seed=seed + 1)
            st["load"] = f
            plain["rates"].append(st)
    out["plain_baseline"] = plain
    return out


def uniform_leg(steps: int):
    """The 256-surface bicubic batch (16x16 control points, 128x128 samples
    each) through the uniform-batch calls -- the paper's
    surface(ctrl, w, ku, kv, p, q, uv) and its backward -- with all four
    gradients; one step (forward + backward) is captured as a HIP graph and
    replayed, the MALL flushed before each step outside its events.  Parity
    on every surface of the timed outputs."""
    import torch
    from paper_2104_14547_amd import api
    from paper_2104_14547_amd import workloads as W
    b = W.batch_bicubic(1)
    b.upstream = np.random.Generator(np.random.PCG64(9)).uniform(-0.1, 0.1, b.n_pts_floats).astype(np.float32)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    B, p, q, nc, ns = b.n, 3, 3, 16, 128
    ctrl, w = T(b.ctrl.reshape(B, nc, nc, 3)), T(b.w.reshape(B, nc, nc))
    ku, kv = T(b.ku.reshape(B, -1)), T(b.kv.reshape(B, -1))
    us = T(b.surface(0)["us"])
    vs = T(b.surface(0)["vs"])
    g = T(b.upstream.reshape(B, ns, ns, 3))
    pts = torch.empty((B, ns, ns, 3), dtype=torch.float32, device=dev)
    grads = [None]

    def body():
        api.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, out=pts)
        grads[0] = api.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, g)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body()
    torch.cuda.synchronize()
    flush = make_flush(torch, dev)
    ms = timed_steps(torch, graph.replay, steps, flush=flush)
    del flush
    par = parity_all(b, pts.reshape(-1).cpu().numpy(), [x.reshape(-1).cpu().numpy() for x in grads[0]])
    ms_step = float(np.mean(ms))
    ab = algorithmic_bytes(b.shapes)
    return {"workload": b.name, "api": "uniform batch (nurbs_surface_fwd / nurbs_surface_bwd), HIP graph",
            "points": b.n_points, "steps": steps, "ms_per_step": ms_step,
            "pts_per_s": b.n_points / (ms_step * 1e-3) if par["pass"] else None,
            "step_algorithmic_GBs": (ab["fwd"] + ab["bwd"] + ab["fin"]) / (ms_step * 1e-3) / 1e9,
            "parity": par}


# VALU issue peak in lane-instructions/s without packed FP32: 256 CUs x 4 SIMDs x 16 lanes per clock x
# 2.4 GHz (a wave64 instruction every 4 cycles per SIMD).  The published 157.3 TFLOP/s FP32 vector rate is
# this rate x 2 flops per FMA x 2 for packed FP32 (two values per lane per instruction), which the library
# does not use; the 78.6 TFLOP/s FP64 vector rate is the same 39.3 T FMA/s x 2 flops.
VALU_PEAK_INSTR = 256 * 4 * 16 * 2.4e9


def _ev(torch):
    return torch.cuda.Event(enable_timing=True)


def curve_leg(steps: int):
    """16384 cubic space curves, 32 control points, 1024 shared samples each,
    through nurbs_curve_fwd / nurbs_curve_bwd (points, weights and knots):
    per-call HIP events on the launch stream, the MALL flushed before each
    step outside the events; parity of the timed outputs on 64 curves."""
    import torch
    from paper_2104_14547_amd import _native as N
    from paper_2104_14547_amd import api
    from paper_2104_14547_amd import workloads as W
    from oracle import oracle as O
    cb = W.curve_batch(seed=8, B=16384, p=3, nc=32, ns=1024, dim=3)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctrl, w, kn, us, g = T(cb.ctrl), T(cb.w), T(cb.knots), T(cb.us), T(cb.upstream)
    B, p, nc, ns, dim = cb.B, cb.p, cb.nc, cb.ns, cb.dim
    ctx = api.context(0)
    pts = torch.empty((B, ns, dim), dtype=torch.float32, device=dev)
    gc, gw, gk = torch.empty_like(ctrl), torch.empty_like(w), torch.empty_like(kn)
    ws_n = __import__("ctypes").c_size_t()
    api._check(N.lib().nurbs_curve_ws_bytes(ctx.handle, B, p, nc, dim, ns, 7, __import__("ctypes").byref(ws_n)))
    ws = torch.empty(max(ws_n.value, 256), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream

    def fwd():
        api._check(N.lib().nurbs_curve_fwd(ctx.handle, B, p, nc, dim, ctrl.data_ptr(), w.data_ptr(), kn.data_ptr(), ns,
                                           us.data_ptr(), 1, pts.data_ptr(), None, None, 0, st), ctx.handle)

    def bwd():
        api._check(N.lib().nurbs_curve_bwd(ctx.handle, B, p, nc, dim, ctrl.data_ptr(), w.data_ptr(), kn.data_ptr(), ns,
                                           us.data_ptr(), 1, g.data_ptr(), gc.data_ptr(), gw.data_ptr(), gk.data_ptr(),
                                           7, ws.data_ptr(), ws.numel(), st), ctx.handle)

    for _ in range(3):
        fwd()
        bwd()
    flush = make_flush(torch, dev)
    ev = [(_ev(torch), _ev(torch), _ev(torch)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b, c in ev:
        evict_mall(torch, flush)
        a.record()
        fwd()
        b.record()
        bwd()
        c.record()
    torch.cuda.synchronize()
    del flush
    tf = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    tb = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    npts, nU = B * ns, nc + p + 1
    per_curve = 4 * (dim + 1) * nc + 4 * nU  # control points + weights, knots
    bytes_fwd = 4 * dim * npts + B * per_curve + 4 * ns
    bytes_bwd = 4 * dim * npts + 2 * B * per_curve + 4 * ns
    # parity of the timed outputs on 64 curves
    sel = np.arange(0, B, B // 64)
    sub = W.CurveBatch(name="sub", p=p, nc=nc, ns=ns, dim=dim, ctrl=cb.ctrl[sel], w=cb.w[sel], knots=cb.knots[sel],
                       us=cb.us, upstream=cb.upstream[sel])

    class _P:
        shapes = np.array([[p, nc, ns, dim]] * len(sel), np.int32)
        offsets = np.array([[c * nc * dim, c * nc, c * nU, c * ns, c * ns * dim] for c in range(len(sel))], np.int64)
        ctrl, w, knots = sub.ctrl.ravel(), sub.w.ravel(), sub.knots.ravel()
        us = np.broadcast_to(sub.us, (len(sel), ns)).ravel()
    S_or = O.curve_fwd(_P).reshape(len(sel), ns, dim)
    G_or = O.curve_bwd(_P, sub.upstream.astype(np.float64).ravel())
    got = pts.cpu().numpy()[sel].astype(np.float64)
    diag = np.linalg.norm(S_or.max(1) - S_or.min(1), axis=1)
    perr = float((np.linalg.norm(got - S_or, axis=2).max(1) / diag).max())
    gerr = 0.0
    for t, ref in zip((gc, gw, gk), G_or):
        a = t.cpu().numpy()[sel].reshape(len(sel), -1).astype(np.float64)
        r = ref.reshape(len(sel), -1)
        gerr = max(gerr, float((np.abs(a - r).max(1) / np.abs(r).max(1)).max()))
    ok = perr <= 1e-5 and gerr <= 1e-4
    dom, t_dom, b_dom = ("k_curve_bwd", tb, bytes_bwd) if tb >= tf else ("k_curve_fwd", tf, bytes_fwd)
    ach = b_dom / (t_dom * 1e-3) / 1e9
    return {"workload": cb.name, "api": "nurbs_curve_fwd / nurbs_curve_bwd (CTRL|W|KU)", "points": npts,
            "steps": steps, "fwd_ms": tf, "bwd_ms": tb,
            "pts_per_s": npts / ((tf + tb) * 1e-3) if ok else None,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes": b_dom},
            "fwd_GBs": bytes_fwd / (tf * 1e-3) / 1e9, "bwd_GBs": bytes_bwd / (tb * 1e-3) / 1e9,
            "parity": {"curves": int(len(sel)), "max_point_err_rel_bbox": perr, "max_grad_err_rel_inf": gerr,
                       "pass": ok}}


def uv_leg(steps: int):
    """64 bicubic 16x16 surfaces, each evaluated at 65536 scattered (u, v)
    pairs in random order (nurbs_surface_uv_fwd / nurbs_surface_uv_bwd, all
    four gradients): HIP events on the launch stream, MALL flushed before each
    step outside the events; parity on 4 surfaces of the timed outputs."""
    import ctypes
    import torch
    from paper_2104_14547_amd import _native as N
    from paper_2104_14547_amd import api
    from paper_2104_14547_amd import workloads as W
    from oracle import oracle as O
    ub = W.uv_batch(seed=9, B=64, p=3, q=3, nu_c=16, nv_c=16, npts=65536)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctrl, w, ku, kv, uv, g = T(ub.ctrl), T(ub.w), T(ub.ku), T(ub.kv), T(ub.uv), T(ub.upstream)
    B, p, q, nc, npts = ub.B, 3, 3, 16, ub.npts
    ctx = api.context(0)
    pts = torch.empty((B, npts, 3), dtype=torch.float32, device=dev)
    gc, gw, gu, gv = (torch.empty_like(x) for x in (ctrl, w, ku, kv))
    ws_n = ctypes.c_size_t()
    api._check(N.lib().nurbs_surface_uv_ws_bytes(ctx.handle, B, p, q, nc, nc, npts, 15, ctypes.byref(ws_n)))
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream

    def fwd():
        api._check(N.lib().nurbs_surface_uv_fwd(ctx.handle, B, p, q, nc, nc, ctrl.data_ptr(), w.data_ptr(),
                                                ku.data_ptr(), kv.data_ptr(), npts, uv.data_ptr(), 0,
                                                pts.data_ptr(), None, None, None, 0, st), ctx.handle)

    def bwd():
        api._check(N.lib().nurbs_surface_uv_bwd(ctx.handle, B, p, q, nc, nc, ctrl.data_ptr(), w.data_ptr(),
                                                ku.data_ptr(), kv.data_ptr(), npts, uv.data_ptr(), 0, g.data_ptr(),
                                                gc.data_ptr(), gw.data_ptr(), gu.data_ptr(), gv.data_ptr(), 15,
                                                ws.data_ptr(), ws.numel(), st), ctx.handle)

    for _ in range(3):
        fwd()
        bwd()
    flush = make_flush(torch, dev)
    ev = [(_ev(torch), _ev(torch), _ev(torch)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b, c in ev:
        evict_mall(torch, flush)
        a.record()
        fwd()
        b.record()
        bwd()
        c.record()
    torch.cuda.synchronize()
    del flush
    tf = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    tb = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    n = B * npts
    per_surf = 16 * nc * nc + 4 * 2 * (nc + p + 1)
    bytes_fwd = 20 * n + B * per_surf
    bytes_bwd = 20 * n + 2 * B * per_surf
    perr = gerr = 0.0
    for b in range(0, B, B // 4):
        S = O.scattered_fwd(ub.ctrl[b], ub.w[b], ub.ku[b], ub.kv[b], p, q, ub.uv[b])
        diag = np.linalg.norm(S.max(0) - S.min(0))
        perr = max(perr, float(np.linalg.norm(pts[b].cpu().numpy() - S, axis=1).max() / diag))
        ref = O.scattered_bwd(ub.ctrl[b], ub.w[b], ub.ku[b], ub.kv[b], p, q, ub.uv[b],
                              ub.upstream[b].astype(np.float64))
        for t, r in zip((gc, gw, gu, gv), ref):
            gerr = max(gerr, float(np.abs(t[b].cpu().numpy().ravel() - r.ravel()).max() / np.abs(r).max()))
    ok = perr <= 1e-5 and gerr <= 1e-4
    dom, t_dom, b_dom = ("k_uv_acc+k_uv_max+k_uv_fin", tb, bytes_bwd) if tb >= tf else ("k_uv_fwd", tf, bytes_fwd)
    ach = b_dom / (t_dom * 1e-3) / 1e9
    return {"workload": ub.name, "api": "nurbs_surface_uv_fwd / nurbs_surface_uv_bwd (all gradients)", "points": n,
            "steps": steps, "fwd_ms": tf, "bwd_ms": tb, "pts_per_s": n / ((tf + tb) * 1e-3) if ok else None,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes": b_dom},
            "fwd_GBs": bytes_fwd / (tf * 1e-3) / 1e9, "bwd_GBs": bytes_bwd / (tb * 1e-3) / 1e9,
            "parity": {"surfaces": 4, "max_point_err_rel_bbox": perr, "max_grad_err_rel_inf": gerr, "pass": ok}}


def chamfer_leg(steps: int):
    """Chamfer and Hausdorff distances and their gradients between 16384
    evaluated points and a 16384-point target cloud (nurbs_chamfer), and the
    brute-force nearest-neighbour search alone (nurbs_nearest), with HIP
    events on the launch stream; parity against the oracle on the timed
    outputs."""
    import ctypes
    import torch
    from paper_2104_14547_amd import _native as N
    from paper_2104_14547_amd import api
    from paper_2104_14547_amd import workloads as W
    from oracle import oracle as O
    n = m = 16384
    P, Q = W.point_sets(seed=6, B=1, n=n, m=m, dim=3)
    dev = torch.device("cuda", 0)
    Pt, Qt = (torch.from_numpy(x).to(dev) for x in (P, Q))
    ctx = api.context(0)
    ws_n = ctypes.c_size_t()
    api._check(N.lib().nurbs_chamfer_ws_bytes(ctx.handle, 1, n, m, ctypes.byref(ws_n)))
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev)
    out = torch.empty(2, dtype=torch.float32, device=dev)
    gcd, ghd = torch.empty_like(Pt), torch.empty_like(Pt)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    d2 = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream().cuda_stream

    def full():
        api._check(N.lib().nurbs_chamfer(ctx.handle, 1, 3, Pt.data_ptr(), n, Qt.data_ptr(), m, out.data_ptr(),
                                         gcd.data_ptr(), ghd.data_ptr(), ws.data_ptr(), ws.numel(), st), ctx.handle)

    def nn():
        api._check(N.lib().nurbs_nearest(ctx.handle, 1, 3, Pt.data_ptr(), n, Qt.data_ptr(), m, idx.data_ptr(),
                                         d2.data_ptr(), ws.data_ptr(), ws.numel(), st), ctx.handle)

    for _ in range(2):
        full()
        nn()
    ev = [(_ev(torch), _ev(torch), _ev(torch)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b, c in ev:
        a.record()
        full()
        b.record()
        nn()
        c.record()
    torch.cuda.synchronize()
    t_full = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    t_nn = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    cd, hd, rg_cd, rg_hd = O.chamfer_hausdorff(P[0], Q[0])
    ri, rd = O.nearest(P[0], Q[0])
    o = out.cpu().numpy().astype(np.float64)
    gerr = max(float(np.abs(gcd.cpu().numpy() - rg_cd).max() / np.abs(rg_cd).max()),
               float(np.abs(ghd.cpu().numpy() - rg_hd).max() / np.abs(rg_hd).max()))
    nn_exact = bool((idx.cpu().numpy() == ri).all() and (d2.cpu().numpy() == rd).all())
    ok = nn_exact and abs(o[0] - cd) <= 1e-5 * cd and abs(o[1] - hd) <= 1e-5 * hd and gerr <= 1e-4
    instr = 9  # per pair: 3 sub, 1 mul, 2 fma, 1 compare, 2 selects
    ach = n * m * instr / (t_nn * 1e-3)
    return {"workload": f"chamfer_hausdorff_{n}x{m}_3d", "api": "nurbs_chamfer (CD, HD, both gradients); nurbs_nearest",
            "pairs_per_nearest": n * m, "steps": steps, "chamfer_ms": t_full, "nearest_ms": t_nn,
            "pair_evals_per_s": 2 * n * m / (t_full * 1e-3) if ok else None,
            "roofline": {"bound": "alu", "kernel": "k_nn+k_nn_merge (nurbs_nearest)", "achieved": ach / 1e12,
                         "peak": VALU_PEAK_INSTR / 1e12,
                         "unit": "T lane-instr/s", "frac": ach / VALU_PEAK_INSTR,
                         "instr_per_pair": instr},
            "parity": {"nearest_bit_exact": nn_exact, "cd_rel_err": abs(o[0] - cd) / cd,
                       "hd_rel_err": abs(o[1] - hd) / hd, "max_grad_err_rel_inf": gerr, "pass": ok}}


def fit_leg(steps: int):
    """The fitting loop (64x64 bicubic net, 512x512 samples of
    z = sin 3x cos 3y, Adam lr 1e-2), one HIP graph launch per step, in three
    variants: points, weights and knots trained; knots fixed with the span and
    basis tables built once (the fixed-knot layer); knots fixed, basis
    evaluated every step."""
    import torch
    from paper_2104_14547_amd import workloads as W
    from paper_2104_14547_amd.fit import SurfaceFit
    b = W.fit_target(2)
    d = b.surface(0)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = {"workload": b.name, "steps": steps,
           "note": "whole step (fwd, dL/dS, bwd, Adam, projections) replayed as one HIP graph"}
    for name, kw in (("knots_trained", dict(train_knots=True)),
                     ("fixed_knots_tables", dict(train_knots=False, cached_basis=True)),
                     ("fixed_knots_no_tables", dict(train_knots=False, cached_basis=False))):
        f = SurfaceFit(T(d["ctrl"]), T(d["w"]), T(d["ku"]), T(d["kv"]), d["p"], d["q"], T(d["us"]), T(d["vs"]),
                       T(d["target"]), lr=1e-2, graph=True, **kw)
        l0 = f.loss()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"step_ms": dt / steps * 1e3, "pts_per_s": b.n_points * steps / dt, "loss_start": l0,
                     "loss_end": f.loss(), "tiles": list(f.tiling)}
    return out


def copy_calibration(torch, dev, mib: int, reps: int = 3):
    """A plain copy of known size: each launch reads and writes exactly
    mib MiB, so what the FETCH_SIZE / WRITE_SIZE counters report for it gives
    the factor that turns those counters into HBM bytes.  An elementwise
    kernel (x * 1) rather than copy_, which may go to a DMA engine."""
    n = mib * 2**20 // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 4, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="uneven_batch", choices=["uneven_batch", "batch_bicubic"])
    ap.add_argument("--cpu-sample", type=int, default=4096, help="surfaces timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="default tiles instead of the autotuned ones")
    ap.add_argument("--tiles", default="", metavar="FWD,BWD",
                    help="fixed sample points per forward,backward tile (skips the autotuner)")
    ap.add_argument("--schedule", default="static", choices=["static", "dynamic"],
                    help="tile schedule with --tiles")
    ap.add_argument("--served-requests", type=int, default=20000,
                    help="requests per arrival rate in the served leg (0: skip it)")
    ap.add_argument("--fit-steps", type=int, default=500, help="steps of the fitting leg (0: skip it)")
    ap.add_argument("--uniform-steps", type=int, default=20,
                    help="steps of the 256-surface bicubic uniform-batch leg (0: skip it)")
    ap.add_argument("--curve-steps", type=int, default=20, help="steps of the curve leg (0: skip it)")
    ap.add_argument("--uv-steps", type=int, default=10, help="steps of the scattered-pair leg (0: skip it)")
    ap.add_argument("--chamfer-steps", type=int, default=10, help="steps of the Chamfer/Hausdorff leg (0: skip it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (scale for HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2104_14547_amd as nd
    from paper_2104_14547_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        copy_calibration(torch, dev, args.copy_calibration)
        return
    t0 = time.perf_counter()
    if args.workload == "uneven_batch":
        batch = W.uneven_batch(3)
    else:
        batch = W.batch_bicubic(1)
        batch.upstream = np.random.Generator(np.random.PCG64(9)).uniform(
            -0.1, 0.1, batch.n_pts_floats).astype(np.float32)
    log(f"[bench] workload {batch.name}: {batch.n} surfaces, {batch.n_points} points "
        f"(generated in {time.perf_counter() - t0:.1f} s)")

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inputs = [T(getattr(batch, k)) for k in ("ctrl", "w", "ku", "kv", "us", "vs")]
    upstream = T(batch.upstream)
    sched = {"dynamic": nd.api.N.NURBS_SCHED_DYNAMIC, "static": nd.api.N.NURBS_SCHED_STATIC}
    if args.tiles:
        tf, tb = (int(x) for x in args.tiles.split(","))
        ctx = nd.api.Context(0)
        ctx.set_tiling(tf, tb)
        ctx.set_schedule(sched[args.schedule])
        plan = nd.SurfaceBatch(batch.shapes, batch.offsets, device=0, ctx=ctx)
        tune = {"chosen": {"schedule": args.schedule, "fwd_tile_points": tf, "bwd_tile_points": tb}, "fixed": True}
    elif args.no_autotune:
        plan, tune = nd.SurfaceBatch(batch.shapes, batch.offsets, device=0), None
    else:
        t1 = time.perf_counter()
        plan, tune = nd.api.autotune(batch.shapes, batch.offsets, inputs, upstream, device=0)
        log(f"[bench] autotune {tune} ({time.perf_counter() - t1:.1f} s)")
    info = plan.info()
    pts = torch.empty(plan.n_pts_floats, dtype=torch.float32, device=dev)
    grads = tuple(torch.empty_like(x) for x in inputs[:4])
    plan.workspace()
    log(f"[bench] plan: {info}, workspace {plan.ws_bytes / 2**20:.1f} MiB")

    def step():
        plan.forward(*inputs, out=pts)
        plan.backward(*inputs, upstream, out=grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # back to back, for reference: the MALL (256 MB) may still hold part of
    # the previous step's data
    t_bb = timed_steps(torch, step, args.steps, flush=None)
    # the timed steps: before each, a 512 MB scratch write and a 512 MB read
    # evict the caches and are waited for, outside the events that time the
    # step, so every step reads its inputs from HBM
    flush = make_flush(torch, dev)
    plan.set_timing(args.steps)
    step_ms = timed_steps(torch, step, args.steps, flush=flush)
    kf, kb, kg, kz = plan.read_timing()
    plan.set_timing(0)
    # for context, the same step captured once as a HIP graph and replayed
    # (launch gaps gone), same eviction; the kernels' own durations cannot be
    # read from events recorded inside a replay, so `value` and the roofline
    # stay with the eager steps above
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    graph_ms = timed_steps(torch, graph.replay, args.steps, flush=flush)
    del graph
    del flush
    ms_step = float(np.mean(step_ms))
    value = batch.n_points / (ms_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step (MALL flushed), {value:.4e} pts/s; "
        f"back to back {np.mean(t_bb):.4f} ms/step; graph replay {np.mean(graph_ms):.4f} ms/step; "
        f"kernels fwd {kf.mean():.4f} ms, bwd {kb.mean():.4f} ms, gather {kg.mean():.4f} ms, "
        f"finalize {kz.mean():.4f} ms")

    ab = algorithmic_bytes(batch.shapes)
    avg = {"fwd": float(kf.mean()), "bwd": float(kb.mean()), "gat": float(kg.mean()), "fin": float(kz.mean())}
    names = {"fwd": "k_fwd_plan", "bwd": "k_bwd_plan", "gat": "k_gat_plan", "fin": "k_fin_plan"}
    # the gather moves no algorithmic bytes (workspace only): the roofline kernel is one of the others
    dom = max((k for k in avg if ab[k] > 0), key=avg.get)
    achieved = ab[dom] / (avg[dom] * 1e-3) / 1e9
    kernels = {names[k]: {"avg_ms": avg[k], "algorithmic_bytes": ab[k],
                          "achieved_GBs": ab[k] / (avg[k] * 1e-3) / 1e9} for k in avg}
    chosen = tune["chosen"] if tune else {"schedule": "static", "fwd_tile_points": 16384, "bwd_tile_points": 16384}
    traffic = traffic_for(names[dom], args.workload, chosen)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": batch.name, "surfaces": batch.n, "points": ab["points"],
                   "control_points": ab["control_points"], "degrees": "p,q in 1..5",
                   "launches_per_step": 4,
                   "tiles": chosen},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernels": kernels,
        "step_algorithmic_GBs": (ab["fwd"] + ab["bwd"] + ab["fin"]) / (ms_step * 1e-3) / 1e9,
        "timing": {"step_ms": "mean of per-step HIP events; before each step a 512 MB scratch write and a "
                              "512 MB read evict the caches (the read leaves them clean) and are waited for "
                              "(host synchronisation), outside the events",
                   "back_to_back_ms_per_step": float(np.mean(t_bb)),
                   "back_to_back_pts_s": batch.n_points / (float(np.mean(t_bb)) * 1e-3),
                   "graph_replay_ms_per_step": float(np.mean(graph_ms)),
                   "graph_replay_pts_s": batch.n_points / (float(np.mean(graph_ms)) * 1e-3)},
    }
    if tune and not tune.get("fixed"):
        result["autotune_ms"] = {d: {str(k): v for k, v in tune[d].items()} for d in ("fwd", "bwd")}
    if not args.no_parity:
        t1 = time.perf_counter()
        result["parity"] = parity_all(batch, pts.cpu().numpy(), [g.cpu().numpy() for g in grads])
        log(f"[bench] parity {result['parity']} ({time.perf_counter() - t1:.1f} s)")
        if not result["parity"]["pass"]:
            # a throughput at failed parity is no measurement
            result["value"] = None
            log("[bench] PARITY FAILED: value withheld")
    if args.uniform_steps > 0:
        t1 = time.perf_counter()
        result["batch_bicubic"] = uniform_leg(args.uniform_steps)
        log(f"[bench] batch_bicubic {result['batch_bicubic']} ({time.perf_counter() - t1:.1f} s)")
    if args.curve_steps > 0:
        t1 = time.perf_counter()
        result["curves"] = curve_leg(args.curve_steps)
        log(f"[bench] curves {result['curves']} ({time.perf_counter() - t1:.1f} s)")
    if args.uv_steps > 0:
        t1 = time.perf_counter()
        result["scattered_uv"] = uv_leg(args.uv_steps)
        log(f"[bench] scattered_uv {result['scattered_uv']} ({time.perf_counter() - t1:.1f} s)")
    if args.chamfer_steps > 0:
        t1 = time.perf_counter()
        result["chamfer"] = chamfer_leg(args.chamfer_steps)
        log(f"[bench] chamfer {result['chamfer']} ({time.perf_counter() - t1:.1f} s)")
    if args.fit_steps > 0:
        t1 = time.perf_counter()
        result["fit"] = fit_leg(args.fit_steps)
        log(f"[bench] fit {result['fit']} ({time.perf_counter() - t1:.1f} s)")
    if args.served_requests > 0:
        t1 = time.perf_counter()
        result["served"] = served_leg(batch, args.served_requests)
        log(f"[bench] served {result['served']} ({time.perf_counter() - t1:.1f} s)")
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        result["cpu_baseline"] = cpu_baseline(batch, args.cpu_sample)
        log(f"[bench] cpu baseline {result['cpu_baseline']['value']:.4e} pts/s "
            f"({time.perf_counter() - t1:.1f} s)")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
