#!/usr/bin/env python
"""Throughput of batched NURBS surface evaluation + adjoint on one MI355X.

Workload (default): the uneven batch -- 4096 surfaces, degrees p, q in 1..5,
control sides 4..48 and sample sides 16..256 (log-uniform), non-uniform
clamped knots with 10% repeated interior knots -- run as one ragged plan:
one persistent forward launch, one persistent backward launch and the
per-surface finalize.  A step is forward + backward (all four gradients)
over the whole batch with every input resident in HBM; the upstream
gradient dL/dS is a fixed synthetic array (see workloads.uneven_batch).

Prints ONE JSON line: metric, value (surface points per second of
forward + backward), roofline of the dominant kernel (algorithmic bytes per
launch / its average duration, from HIP events recorded around each kernel
during the timed steps), the FP64 oracle's throughput on a bounded sample of
the same batch (cpu_baseline) and the parity errors of the timed outputs on
sampled surfaces.
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


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2104_14547_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(shapes):
    """Bytes the method must move, per kernel (float32).

    forward : write S (12 B/pt), read P and W (16 B/control point), read the
              samples (4 B each) and knots (4 B each);
    backward: read dL/dS (12 B/pt), read P and W, samples and knots;
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
            "fin": 16 * cps + 4 * kn}


def traffic_for(kernel: str, workload: str, tiles: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources at the same tiling; else None."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    if rec.get("tiles") != tiles:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def timed_steps(torch, step, n: int, flush=None):
    """Run ``step`` n times between HIP events on the current stream; with
    ``flush`` (a large device buffer), fill it before each step, outside the
    events.  Returns the per-step times in ms."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        if flush is not None:
            flush.fill_(0.0)
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
    loop saturation, then Poisson arrivals at 0.5x, 0.8x and 1.0x of it, and
    the per-request plain-launch baseline at the same rates (fewer requests:
    it saturates far earlier)."""
    from paper_2104_14547_amd.serve import PlainServer, Server, make_requests, run_load
    reqs = make_requests(batch, n_req, seed=seed)
    out = {"requests_per_rate": n_req, "rates": []}
    with Server(batch, slot_bytes=1 << 30, n_slots=3, max_requests=512) as srv:
        run_load(srv, reqs[: min(200, n_req)], rate=None)  # warm-up
        sat, _ = run_load(srv, reqs, rate=None)
        out["saturation_req_s"] = sat["req_per_s"]
        out["saturation_pts_s"] = sat["pts_per_s"]
        for f in (0.5, 0.8, 1.0):
            st, _ = run_load(srv, reqs, rate=f * sat["req_per_s"], seed=seed + 1)
            st["load"] = f
            out["rates"].append(st)
        out["batches"] = srv.batches
    n_plain = min(n_req, 400)
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
    flush = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
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


def fit_leg(steps: int):
    """The fitting loop (64x64 bicubic net, 512x512 samples of
    z = sin 3x cos 3y, Adam lr 1e-2 on points, weights and knots), one HIP
    graph launch per step."""
    import torch
    from paper_2104_14547_amd import workloads as W
    from paper_2104_14547_amd.fit import SurfaceFit
    b = W.fit_target(2)
    d = b.surface(0)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    f = SurfaceFit(T(d["ctrl"]), T(d["w"]), T(d["ku"]), T(d["kv"]), d["p"], d["q"], T(d["us"]), T(d["vs"]),
                   T(d["target"]), lr=1e-2, train_knots=True, graph=True)
    l0 = f.loss()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": b.name, "steps": steps, "step_ms": dt / steps * 1e3,
            "pts_per_s": b.n_points * steps / dt, "loss_start": l0, "loss_end": f.loss(),
            "note": "whole step (fwd, dL/dS, bwd, Adam, projections) replayed as one HIP graph"}


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
    ap.add_argument("--served-requests", type=int, default=3000,
                    help="requests per arrival rate in the served leg (0: skip it)")
    ap.add_argument("--fit-steps", type=int, default=500, help="steps of the fitting leg (0: skip it)")
    ap.add_argument("--uniform-steps", type=int, default=20,
                    help="steps of the 256-surface bicubic uniform-batch leg (0: skip it)")
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
    if args.tiles:
        tf, tb = (int(x) for x in args.tiles.split(","))
        ctx = nd.api.Context(0)
        ctx.set_tiling(tf, tb)
        plan = nd.SurfaceBatch(batch.shapes, batch.offsets, device=0, ctx=ctx)
        tune = {"chosen": {"fwd_tile_points": tf, "bwd_tile_points": tb}, "fixed": True}
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
    # the timed steps: before each, a 512 MB fill evicts the MALL, outside the
    # events that time the step, so every step reads its inputs from HBM
    flush = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
    plan.set_timing(args.steps)
    step_ms = timed_steps(torch, step, args.steps, flush=flush)
    kf, kb, kz = plan.read_timing()
    plan.set_timing(0)
    del flush
    ms_step = float(np.mean(step_ms))
    value = batch.n_points / (ms_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step (MALL flushed), {value:.4e} pts/s; "
        f"back to back {np.mean(t_bb):.4f} ms/step; "
        f"kernels fwd {kf.mean():.4f} ms, bwd {kb.mean():.4f} ms, finalize {kz.mean():.4f} ms")

    ab = algorithmic_bytes(batch.shapes)
    avg = {"fwd": float(kf.mean()), "bwd": float(kb.mean()), "fin": float(kz.mean())}
    names = {"fwd": "k_fwd_plan", "bwd": "k_bwd_plan", "fin": "k_fin_plan"}
    dom = max(avg, key=avg.get)
    achieved = ab[dom] / (avg[dom] * 1e-3) / 1e9
    kernels = {names[k]: {"avg_ms": avg[k], "algorithmic_bytes": ab[k],
                          "achieved_GBs": ab[k] / (avg[k] * 1e-3) / 1e9} for k in avg}
    chosen = tune["chosen"] if tune else {"fwd_tile_points": 16384, "bwd_tile_points": 16384}
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
                   "launches_per_step": 3,
                   "tiles": chosen},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernels": kernels,
        "step_algorithmic_GBs": (ab["fwd"] + ab["bwd"] + ab["fin"]) / (ms_step * 1e-3) / 1e9,
        "timing": {"step_ms": "mean of per-step HIP events; a 512 MB fill evicts the MALL before each step, "
                              "outside the events",
                   "back_to_back_ms_per_step": float(np.mean(t_bb)),
                   "back_to_back_pts_s": batch.n_points / (float(np.mean(t_bb)) * 1e-3)},
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
