"""PyTorch-facing API over libnurbsdiff.

PyTorch supplies device memory and streams; every step of the computation
runs in the library's HIP kernels.  Shapes follow the paper's statement of the
problem, surface(ctrl_pts, weights, knot_u, knot_v, p, q, uv) -> points
(Sec. 3.1, eq. ForwardEvaluation), and its backward (Sec. 3.2).
"""
from __future__ import annotations

import ctypes
import threading

import numpy as np
import torch

from . import _native as N


class NurbsError(RuntimeError):
    """A non-zero status from libnurbsdiff."""

    def __init__(self, code: int, message: str):
        self.code = int(code)
        super().__init__(f"{N.status_string(code)} ({code}): {message}")


def _check(rc: int, ctx_handle=None):
    if rc != N.NURBS_OK:
        msg = N.lib().nurbs_last_error(ctx_handle).decode()
        raise NurbsError(rc, msg)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need_cuda_f32(name, t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


class Context:
    """One libnurbsdiff context (device ordinal, flags, last error)."""

    def __init__(self, device: int | None = None, validate: bool = False):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(N.lib().nurbs_ctx_create(self.device, ctypes.byref(h)))
        self.handle = h
        self.flags = 0
        if validate:
            self.set_flags(N.NURBS_VALIDATE)

    def set_flags(self, flags: int):
        _check(N.lib().nurbs_ctx_set_flags(self.handle, int(flags)), self.handle)
        self.flags = int(flags)

    @property
    def validate(self) -> bool:
        return bool(self.flags & N.NURBS_VALIDATE)

    def read_device_error(self, ws, device=None) -> int:
        code = ctypes.c_int()
        _check(N.lib().nurbs_read_device_error(_ptr(ws), _stream(ws.device), ctypes.byref(code)))
        return code.value

    def set_knot_sigma(self, sigma: float):
        _check(N.lib().nurbs_ctx_set_knot_sigma(self.handle, float(sigma)), self.handle)

    def set_tiling(self, fwd_tile_points: int = 0, bwd_tile_points: int = 0):
        """Target sample points per forward / backward tile of later calls (0: default)."""
        _check(N.lib().nurbs_ctx_set_tiling(self.handle, int(fwd_tile_points), int(bwd_tile_points)), self.handle)
        self.tiling = (int(fwd_tile_points) or 16384, int(bwd_tile_points) or 16384)

    def set_schedule(self, schedule: int):
        """Tile schedule of plans created later on this context
        (NURBS_SCHED_DYNAMIC, the default, or NURBS_SCHED_STATIC)."""
        _check(N.lib().nurbs_ctx_set_schedule(self.handle, int(schedule)), self.handle)
        self.schedule = int(schedule)

    def device_info(self):
        cus, wave = ctypes.c_int(), ctypes.c_int()
        _check(N.lib().nurbs_ctx_device_info(self.handle, ctypes.byref(cus), ctypes.byref(wave)), self.handle)
        return cus.value, wave.value

    def close(self):
        if self.handle:
            N.lib().nurbs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_tls = threading.local()


def context(device: int | None = None) -> Context:
    """The calling thread's default context for ``device``."""
    if device is None:
        device = torch.cuda.current_device()
    cache = getattr(_tls, "ctx", None)
    if cache is None:
        cache = _tls.ctx = {}
    c = cache.get(device)
    if c is None:
        c = cache[device] = Context(device)
    return c


def _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs):
    _need_cuda_f32("ctrl", ctrl)
    for name, t in (("w", w), ("ku", ku), ("kv", kv), ("us", us), ("vs", vs)):
        _need_cuda_f32(name, t)
    if ctrl.dim() == 3:
        ctrl, w, ku, kv = ctrl[None], w[None], ku[None], kv[None]
    if ctrl.dim() != 4 or ctrl.shape[-1] != 3:
        raise ValueError("ctrl must be [B, nu_c, nv_c, 3] or [nu_c, nv_c, 3]")
    B, nu_c, nv_c = (int(x) for x in ctrl.shape[:3])
    if tuple(w.shape) != (B, nu_c, nv_c):
        raise ValueError("w must be [B, nu_c, nv_c]")
    if tuple(ku.shape) != (B, nu_c + p + 1) or tuple(kv.shape) != (B, nv_c + q + 1):
        raise ValueError("knot vectors must be [B, nu_c+p+1] and [B, nv_c+q+1]")
    if us.dim() == 1 and vs.dim() == 1:
        shared = 1
        nu_s, nv_s = int(us.shape[0]), int(vs.shape[0])
    elif us.dim() == 2 and vs.dim() == 2 and us.shape[0] == B and vs.shape[0] == B:
        shared = 0
        nu_s, nv_s = int(us.shape[1]), int(vs.shape[1])
    else:
        raise ValueError("us, vs must both be [n] (shared) or both be [B, n]")
    return ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared


def surface_fwd(ctrl, w, ku, kv, p: int, q: int, us, vs, out=None, ctx: Context | None = None):
    """Points S[B, nu_s, nv_s, 3] of a uniform batch (nurbs_surface_fwd)."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared = _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs)
    ctx = ctx or context(ctrl.device.index)
    if out is None:
        out = torch.empty((B, nu_s, nv_s, 3), dtype=torch.float32, device=ctrl.device)
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_surface_ws_bytes(ctx.handle, B, p, q, nu_c, nv_c, nu_s, nv_s, 0,
                                          ctypes.byref(ws_n)), ctx.handle)
    ws = torch.zeros(ws_n.value, dtype=torch.uint8, device=ctrl.device) if ws_n.value else None
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_fwd(ctx.handle, B, p, q, nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv),
                                     nu_s, nv_s, _ptr(us), _ptr(vs), shared, _ptr(out), _ptr(ws), ws_n.value,
                                     _stream(ctrl.device)), ctx.handle)
    return out[0] if squeeze else out


def surface_derivs(ctrl, w, ku, kv, p: int, q: int, us, vs, want=("pts", "du", "dv", "normals"),
                   ctx: Context | None = None):
    """Points, parametric derivatives dS/du, dS/dv and unit normals of a
    uniform batch (nurbs_surface_derivs).  Returns a dict with the requested
    keys, each [B, nu_s, nv_s, 3] (or [nu_s, nv_s, 3] for one surface)."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared = _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs)
    names = ("pts", "du", "dv", "normals")
    if not want or any(k not in names for k in want):
        raise ValueError(f"want must be a non-empty subset of {names}")
    ctx = ctx or context(ctrl.device.index)
    out = {k: torch.empty((B, nu_s, nv_s, 3), dtype=torch.float32, device=ctrl.device) for k in want}
    ws = torch.zeros(256, dtype=torch.uint8, device=ctrl.device) if ctx.validate else None
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_derivs(ctx.handle, B, p, q, nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv),
                                        nu_s, nv_s, _ptr(us), _ptr(vs), shared,
                                        *[_ptr(out.get(k)) for k in names], _ptr(ws), 0 if ws is None else 256,
                                        _stream(ctrl.device)), ctx.handle)
    return {k: (v[0] if squeeze else v) for k, v in out.items()}


def surface_bwd(ctrl, w, ku, kv, p: int, q: int, us, vs, grad_pts, mask: int = N.NURBS_GRAD_ALL,
                ctx: Context | None = None):
    """(dL/dctrl, dL/dw, dL/dku, dL/dkv) of a uniform batch (nurbs_surface_bwd).
    Entries whose mask bit is clear are None."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared = _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs)
    grad_pts = grad_pts.contiguous()
    if squeeze:
        grad_pts = grad_pts[None]
    _need_cuda_f32("grad_pts", grad_pts)
    if tuple(grad_pts.shape) != (B, nu_s, nv_s, 3):
        raise ValueError("grad_pts must be [B, nu_s, nv_s, 3]")
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    gc = torch.empty_like(ctrl) if mask & N.NURBS_GRAD_CTRL else None
    gw = torch.empty_like(w) if mask & N.NURBS_GRAD_W else None
    gu = torch.empty_like(ku) if mask & N.NURBS_GRAD_KU else None
    gv = torch.empty_like(kv) if mask & N.NURBS_GRAD_KV else None
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_surface_ws_bytes(ctx.handle, B, p, q, nu_c, nv_c, nu_s, nv_s, mask,
                                          ctypes.byref(ws_n)), ctx.handle)
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev) if ws_n.value else None
    if ws is not None and ctx.validate:
        ws[:256].zero_()
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_bwd(ctx.handle, B, p, q, nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv),
                                     nu_s, nv_s, _ptr(us), _ptr(vs), shared, _ptr(grad_pts), _ptr(gc), _ptr(gw),
                                     _ptr(gu), _ptr(gv), int(mask), _ptr(ws), ws_n.value, _stream(dev)),
           ctx.handle)
    res = (gc, gw, gu, gv)
    if squeeze:
        res = tuple(None if r is None else r[0] for r in res)
    return res


# --------------------------------------------------------------------------
# fixed knots: precomputed span and basis tables
# --------------------------------------------------------------------------

def basis_table_bytes(p: int, nx: int) -> int:
    out = ctypes.c_size_t()
    _check(N.lib().nurbs_basis_table_bytes(int(p), int(nx), ctypes.byref(out)))
    return out.value


def basis_table(knots, p: int, x):
    """Span and basis table(s) of the parameters x on the knots
    (nurbs_basis_table_build): knots [n_knots], x [nx] give one table;
    knots [B, n_knots], x [B, nx] (or [nx]) give B tables back to back.
    Returns a uint8 device tensor [B, table_bytes] (B = 1 for one table)."""
    _need_cuda_f32("knots", knots)
    _need_cuda_f32("x", x)
    kn = knots if knots.dim() == 2 else knots[None]
    B, nx = int(kn.shape[0]), int(x.shape[-1])
    xs = x if x.dim() == 2 else x[None].expand(B, nx)
    nb = basis_table_bytes(p, nx)
    out = torch.empty((B, nb), dtype=torch.uint8, device=knots.device)
    st = _stream(knots.device)
    for b in range(B):
        xb = xs[b].contiguous()
        _check(N.lib().nurbs_basis_table_build(_ptr(kn[b]), int(kn.shape[1]), int(p), _ptr(xb), nx,
                                               out[b].data_ptr(), nb, st))
    return out


def _tab_shared(tab_u, tab_v, B):
    if tab_u.dim() != 2 or tab_v.dim() != 2 or tab_u.shape[0] != tab_v.shape[0] or tab_u.shape[0] not in (1, B):
        raise ValueError("tables must be [1, bytes] (shared) or [B, bytes]")
    return 1 if tab_u.shape[0] == 1 else 0


def surface_fwd_tab(ctrl, w, ku, kv, p: int, q: int, us, vs, tab_u, tab_v, out=None, ctx: Context | None = None):
    """Points of a uniform batch on fixed knots from precomputed basis tables
    (nurbs_surface_fwd_tab); tab_u, tab_v from ``basis_table``."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared = _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs)
    ctx = ctx or context(ctrl.device.index)
    if out is None:
        out = torch.empty((B, nu_s, nv_s, 3), dtype=torch.float32, device=ctrl.device)
    ts = _tab_shared(tab_u, tab_v, B)
    ws = torch.zeros(256, dtype=torch.uint8, device=ctrl.device) if ctx.validate else None
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_fwd_tab(ctx.handle, B, p, q, nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv),
                                         nu_s, nv_s, _ptr(us), _ptr(vs), shared, _ptr(tab_u), _ptr(tab_v), ts,
                                         _ptr(out), _ptr(ws), 0 if ws is None else 256, _stream(ctrl.device)),
           ctx.handle)
    return out[0] if squeeze else out


def surface_bwd_tab(ctrl, w, ku, kv, p: int, q: int, us, vs, tab_u, tab_v, grad_pts,
                    mask: int = N.NURBS_GRAD_CTRL | N.NURBS_GRAD_W, ctx: Context | None = None):
    """(dL/dctrl, dL/dw) on fixed knots from precomputed basis tables
    (nurbs_surface_bwd_tab)."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, nu_s, nv_s, shared = _uniform_shapes(ctrl, w, ku, kv, p, q, us, vs)
    grad_pts = grad_pts.contiguous()
    if squeeze:
        grad_pts = grad_pts[None]
    _need_cuda_f32("grad_pts", grad_pts)
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    gc = torch.empty_like(ctrl) if mask & N.NURBS_GRAD_CTRL else None
    gw = torch.empty_like(w) if mask & N.NURBS_GRAD_W else None
    ts = _tab_shared(tab_u, tab_v, B)
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_surface_ws_bytes(ctx.handle, B, p, q, nu_c, nv_c, nu_s, nv_s, mask,
                                          ctypes.byref(ws_n)), ctx.handle)
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev) if ws_n.value else None
    if ws is not None and ctx.validate:
        ws[:256].zero_()
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_bwd_tab(ctx.handle, B, p, q, nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv),
                                         nu_s, nv_s, _ptr(us), _ptr(vs), shared, _ptr(tab_u), _ptr(tab_v), ts,
                                         _ptr(grad_pts), _ptr(gc), _ptr(gw), int(mask), _ptr(ws), ws_n.value,
                                         _stream(dev)), ctx.handle)
    if squeeze:
        return (None if gc is None else gc[0]), (None if gw is None else gw[0])
    return gc, gw


class NurbsSurfaceFn(torch.autograd.Function):
    """Differentiable uniform-batch evaluation; the backward is the library's
    hand-written adjoint (no autograd tape through the kernels)."""

    @staticmethod
    def forward(fctx, ctrl, w, ku, kv, p, q, us, vs):
        pts = surface_fwd(ctrl, w, ku, kv, p, q, us, vs)
        fctx.save_for_backward(ctrl, w, ku, kv, us, vs)
        fctx.pq = (p, q)
        return pts

    @staticmethod
    def backward(fctx, grad_pts):
        ctrl, w, ku, kv, us, vs = fctx.saved_tensors
        p, q = fctx.pq
        need = fctx.needs_input_grad
        mask = (N.NURBS_GRAD_CTRL if need[0] else 0) | (N.NURBS_GRAD_W if need[1] else 0) | \
               (N.NURBS_GRAD_KU if need[2] else 0) | (N.NURBS_GRAD_KV if need[3] else 0)
        if mask == 0:
            return (None,) * 8
        gc, gw, gu, gv = surface_bwd(ctrl, w, ku, kv, p, q, us, vs, grad_pts.contiguous(), mask)
        return gc, gw, gu, gv, None, None, None, None


def surface(ctrl, w, ku, kv, p: int, q: int, us, vs):
    """S = surface(ctrl, w, ku, kv, p, q, us, vs), differentiable in ctrl, w,
    ku and kv (the parameters us, vs get no gradient)."""
    return NurbsSurfaceFn.apply(ctrl.contiguous(), w.contiguous(), ku.contiguous(), kv.contiguous(),
                                int(p), int(q), us.contiguous(), vs.contiguous())


class NurbsSurface(torch.nn.Module):
    """A batch of B surfaces of one shape as trainable parameters."""

    def __init__(self, ctrl, w, ku, kv, p: int, q: int, train_knots: bool = True):
        super().__init__()
        self.p, self.q = int(p), int(q)
        self.ctrl = torch.nn.Parameter(ctrl.detach().clone().contiguous())
        self.w = torch.nn.Parameter(w.detach().clone().contiguous())
        self.ku = torch.nn.Parameter(ku.detach().clone().contiguous(), requires_grad=train_knots)
        self.kv = torch.nn.Parameter(kv.detach().clone().contiguous(), requires_grad=train_knots)

    def forward(self, us, vs):
        return surface(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, us, vs)


# --------------------------------------------------------------------------
# curves
# --------------------------------------------------------------------------

def _curve_shapes(ctrl, w, knots, p, us):
    for name, t in (("ctrl", ctrl), ("w", w), ("knots", knots), ("us", us)):
        _need_cuda_f32(name, t)
    if ctrl.dim() == 2:
        ctrl, w, knots = ctrl[None], w[None], knots[None]
    if ctrl.dim() != 3 or ctrl.shape[-1] not in (2, 3):
        raise ValueError("ctrl must be [B, nc, dim] or [nc, dim] with dim 2 or 3")
    B, nc, dim = (int(x) for x in ctrl.shape)
    if tuple(w.shape) != (B, nc) or tuple(knots.shape) != (B, nc + p + 1):
        raise ValueError("w must be [B, nc] and knots [B, nc+p+1]")
    if us.dim() == 1:
        shared, ns = 1, int(us.shape[0])
    elif us.dim() == 2 and us.shape[0] == B:
        shared, ns = 0, int(us.shape[1])
    else:
        raise ValueError("us must be [ns] (shared) or [B, ns]")
    return ctrl, w, knots, B, nc, dim, ns, shared


def curve_fwd(ctrl, w, knots, p: int, us, derivs: bool = False, ctx: Context | None = None):
    """Points C[B, ns, dim] (and dC/du when ``derivs``) of B curves of one
    shape (nurbs_curve_fwd)."""
    squeeze = ctrl.dim() == 2
    ctrl, w, knots, B, nc, dim, ns, shared = _curve_shapes(ctrl, w, knots, p, us)
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    pts = torch.empty((B, ns, dim), dtype=torch.float32, device=dev)
    du = torch.empty_like(pts) if derivs else None
    ws = torch.zeros(256, dtype=torch.uint8, device=dev) if ctx.validate else None
    ctx.last_ws = ws
    _check(N.lib().nurbs_curve_fwd(ctx.handle, B, int(p), nc, dim, _ptr(ctrl), _ptr(w), _ptr(knots), ns, _ptr(us),
                                   shared, _ptr(pts), _ptr(du), _ptr(ws), 0 if ws is None else 256, _stream(dev)),
           ctx.handle)
    if squeeze:
        pts, du = pts[0], (None if du is None else du[0])
    return (pts, du) if derivs else pts


def curve_bwd(ctrl, w, knots, p: int, us, grad_pts, mask: int = N.NURBS_GRAD_CTRL | N.NURBS_GRAD_W | N.NURBS_GRAD_KU,
              ctx: Context | None = None):
    """(dL/dctrl, dL/dw, dL/dknots) of B curves (nurbs_curve_bwd); entries
    whose mask bit is clear are None."""
    squeeze = ctrl.dim() == 2
    ctrl, w, knots, B, nc, dim, ns, shared = _curve_shapes(ctrl, w, knots, p, us)
    grad_pts = grad_pts.contiguous()
    if squeeze:
        grad_pts = grad_pts[None]
    _need_cuda_f32("grad_pts", grad_pts)
    if tuple(grad_pts.shape) != (B, ns, dim):
        raise ValueError("grad_pts must be [B, ns, dim]")
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    gc = torch.empty_like(ctrl) if mask & N.NURBS_GRAD_CTRL else None
    gw = torch.empty_like(w) if mask & N.NURBS_GRAD_W else None
    gk = torch.empty_like(knots) if mask & N.NURBS_GRAD_KU else None
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_curve_ws_bytes(ctx.handle, B, int(p), nc, dim, ns, int(mask), ctypes.byref(ws_n)),
           ctx.handle)
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev) if ws_n.value else None
    if ws is not None and ctx.validate:
        ws[:256].zero_()
    ctx.last_ws = ws
    _check(N.lib().nurbs_curve_bwd(ctx.handle, B, int(p), nc, dim, _ptr(ctrl), _ptr(w), _ptr(knots), ns, _ptr(us),
                                   shared, _ptr(grad_pts), _ptr(gc), _ptr(gw), _ptr(gk), int(mask), _ptr(ws),
                                   ws_n.value, _stream(dev)), ctx.handle)
    res = (gc, gw, gk)
    if squeeze:
        res = tuple(None if r is None else r[0] for r in res)
    return res


class NurbsCurveFn(torch.autograd.Function):
    """Differentiable curve evaluation with the library's adjoint."""

    @staticmethod
    def forward(fctx, ctrl, w, knots, p, us):
        pts = curve_fwd(ctrl, w, knots, p, us)
        fctx.save_for_backward(ctrl, w, knots, us)
        fctx.p = p
        return pts

    @staticmethod
    def backward(fctx, grad_pts):
        ctrl, w, knots, us = fctx.saved_tensors
        need = fctx.needs_input_grad
        mask = (N.NURBS_GRAD_CTRL if need[0] else 0) | (N.NURBS_GRAD_W if need[1] else 0) | \
               (N.NURBS_GRAD_KU if need[2] else 0)
        if mask == 0:
            return (None,) * 5
        gc, gw, gk = curve_bwd(ctrl, w, knots, fctx.p, us, grad_pts.contiguous(), mask)
        return gc, gw, gk, None, None


def curve(ctrl, w, knots, p: int, us):
    """C = curve(ctrl, w, knots, p, us), differentiable in ctrl, w and knots."""
    return NurbsCurveFn.apply(ctrl.contiguous(), w.contiguous(), knots.contiguous(), int(p), us.contiguous())


# --------------------------------------------------------------------------
# surfaces at scattered (u, v) pairs
# --------------------------------------------------------------------------

def _uv_shapes(ctrl, w, ku, kv, p, q, uv):
    for name, t in (("ctrl", ctrl), ("w", w), ("ku", ku), ("kv", kv), ("uv", uv)):
        _need_cuda_f32(name, t)
    if ctrl.dim() == 3:
        ctrl, w, ku, kv = ctrl[None], w[None], ku[None], kv[None]
    if ctrl.dim() != 4 or ctrl.shape[-1] != 3:
        raise ValueError("ctrl must be [B, nu_c, nv_c, 3] or [nu_c, nv_c, 3]")
    B, nu_c, nv_c = (int(x) for x in ctrl.shape[:3])
    if tuple(w.shape) != (B, nu_c, nv_c) or tuple(ku.shape) != (B, nu_c + p + 1) or \
            tuple(kv.shape) != (B, nv_c + q + 1):
        raise ValueError("w must be [B, nu_c, nv_c], knots [B, nu_c+p+1] and [B, nv_c+q+1]")
    if uv.dim() == 2 and uv.shape[1] == 2:
        shared, npts = 1, int(uv.shape[0])
    elif uv.dim() == 3 and uv.shape[0] == B and uv.shape[2] == 2:
        shared, npts = 0, int(uv.shape[1])
    else:
        raise ValueError("uv must be [npts, 2] (shared) or [B, npts, 2]")
    return ctrl, w, ku, kv, B, nu_c, nv_c, npts, shared


def surface_uv_fwd(ctrl, w, ku, kv, p: int, q: int, uv, derivs: bool = False, ctx: Context | None = None):
    """S [B, npts, 3] at scattered pairs (nurbs_surface_uv_fwd); with
    ``derivs`` also (dS/du, dS/dv)."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, npts, shared = _uv_shapes(ctrl, w, ku, kv, p, q, uv)
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    pts = torch.empty((B, npts, 3), dtype=torch.float32, device=dev)
    du = torch.empty_like(pts) if derivs else None
    dv = torch.empty_like(pts) if derivs else None
    ws = torch.zeros(256, dtype=torch.uint8, device=dev) if ctx.validate else None
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_uv_fwd(ctx.handle, B, int(p), int(q), nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku),
                                        _ptr(kv), npts, _ptr(uv), shared, _ptr(pts), _ptr(du), _ptr(dv), _ptr(ws),
                                        0 if ws is None else 256, _stream(dev)), ctx.handle)
    out = (pts, du, dv)
    if squeeze:
        out = tuple(None if x is None else x[0] for x in out)
    return out if derivs else out[0]


def surface_uv_bwd(ctrl, w, ku, kv, p: int, q: int, uv, grad_pts, mask: int = N.NURBS_GRAD_ALL,
                   ctx: Context | None = None):
    """(dL/dctrl, dL/dw, dL/dku, dL/dkv) at scattered pairs (nurbs_surface_uv_bwd)."""
    squeeze = ctrl.dim() == 3
    ctrl, w, ku, kv, B, nu_c, nv_c, npts, shared = _uv_shapes(ctrl, w, ku, kv, p, q, uv)
    grad_pts = grad_pts.contiguous()
    if squeeze:
        grad_pts = grad_pts[None]
    _need_cuda_f32("grad_pts", grad_pts)
    if tuple(grad_pts.shape) != (B, npts, 3):
        raise ValueError("grad_pts must be [B, npts, 3]")
    ctx = ctx or context(ctrl.device.index)
    dev = ctrl.device
    gc = torch.empty_like(ctrl) if mask & N.NURBS_GRAD_CTRL else None
    gw = torch.empty_like(w) if mask & N.NURBS_GRAD_W else None
    gu = torch.empty_like(ku) if mask & N.NURBS_GRAD_KU else None
    gv = torch.empty_like(kv) if mask & N.NURBS_GRAD_KV else None
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_surface_uv_ws_bytes(ctx.handle, B, int(p), int(q), nu_c, nv_c, npts, int(mask),
                                             ctypes.byref(ws_n)), ctx.handle)
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev) if ws_n.value else None
    if ws is not None and ctx.validate:
        ws[:256].zero_()
    ctx.last_ws = ws
    _check(N.lib().nurbs_surface_uv_bwd(ctx.handle, B, int(p), int(q), nu_c, nv_c, _ptr(ctrl), _ptr(w), _ptr(ku),
                                        _ptr(kv), npts, _ptr(uv), shared, _ptr(grad_pts), _ptr(gc), _ptr(gw),
                                        _ptr(gu), _ptr(gv), int(mask), _ptr(ws), ws_n.value, _stream(dev)),
           ctx.handle)
    res = (gc, gw, gu, gv)
    if squeeze:
        res = tuple(None if r is None else r[0] for r in res)
    return res


class NurbsSurfaceUVFn(torch.autograd.Function):
    """Differentiable evaluation at scattered pairs with the library's adjoint."""

    @staticmethod
    def forward(fctx, ctrl, w, ku, kv, p, q, uv):
        pts = surface_uv_fwd(ctrl, w, ku, kv, p, q, uv)
        fctx.save_for_backward(ctrl, w, ku, kv, uv)
        fctx.pq = (p, q)
        return pts

    @staticmethod
    def backward(fctx, grad_pts):
        ctrl, w, ku, kv, uv = fctx.saved_tensors
        need = fctx.needs_input_grad
        mask = (N.NURBS_GRAD_CTRL if need[0] else 0) | (N.NURBS_GRAD_W if need[1] else 0) | \
               (N.NURBS_GRAD_KU if need[2] else 0) | (N.NURBS_GRAD_KV if need[3] else 0)
        if mask == 0:
            return (None,) * 7
        gc, gw, gu, gv = surface_uv_bwd(ctrl, w, ku, kv, *fctx.pq, uv, grad_pts.contiguous(), mask)
        return gc, gw, gu, gv, None, None, None


def surface_uv(ctrl, w, ku, kv, p: int, q: int, uv):
    """S = surface(ctrl, w, ku, kv, p, q, uv) at scattered pairs uv [npts, 2],
    differentiable in ctrl, w, ku and kv."""
    return NurbsSurfaceUVFn.apply(ctrl.contiguous(), w.contiguous(), ku.contiguous(), kv.contiguous(), int(p),
                                  int(q), uv.contiguous())


# --------------------------------------------------------------------------
# point-set losses
# --------------------------------------------------------------------------

def _sets(P, Q):
    _need_cuda_f32("P", P)
    _need_cuda_f32("Q", Q)
    squeeze = P.dim() == 2
    if squeeze:
        P, Q = P[None], Q[None]
    if P.dim() != 3 or Q.dim() != 3 or P.shape[0] != Q.shape[0] or P.shape[2] != Q.shape[2] or \
            P.shape[2] not in (2, 3):
        raise ValueError("P, Q must be [B, n, dim] and [B, m, dim] (or [n, dim], [m, dim]) with dim 2 or 3")
    return P, Q, int(P.shape[0]), int(P.shape[1]), int(Q.shape[1]), int(P.shape[2]), squeeze


def _cd_ws(ctx, B, n, m, dev):
    ws_n = ctypes.c_size_t()
    _check(N.lib().nurbs_chamfer_ws_bytes(ctx.handle, B, n, m, ctypes.byref(ws_n)), ctx.handle)
    return torch.empty(ws_n.value, dtype=torch.uint8, device=dev)


def nearest(X, Y, ctx: Context | None = None):
    """(idx [B, n] int32, d2 [B, n]) of each X point's nearest Y point (nurbs_nearest)."""
    X, Y, B, n, m, dim, squeeze = _sets(X, Y)
    ctx = ctx or context(X.device.index)
    idx = torch.empty((B, n), dtype=torch.int32, device=X.device)
    d2 = torch.empty((B, n), dtype=torch.float32, device=X.device)
    ws = _cd_ws(ctx, B, n, m, X.device)
    _check(N.lib().nurbs_nearest(ctx.handle, B, dim, _ptr(X), n, _ptr(Y), m, _ptr(idx), _ptr(d2), _ptr(ws),
                                 ws.numel(), _stream(X.device)), ctx.handle)
    return (idx[0], d2[0]) if squeeze else (idx, d2)


def chamfer_hausdorff(P, Q, grads: bool = True, ctx: Context | None = None):
    """(CD [B], HD [B], dCD/dP, dHD/dP) of point sets (nurbs_chamfer)."""
    P, Q, B, n, m, dim, squeeze = _sets(P, Q)
    ctx = ctx or context(P.device.index)
    out = torch.empty((B, 2), dtype=torch.float32, device=P.device)
    gcd = torch.empty_like(P) if grads else None
    ghd = torch.empty_like(P) if grads else None
    ws = _cd_ws(ctx, B, n, m, P.device)
    _check(N.lib().nurbs_chamfer(ctx.handle, B, dim, _ptr(P), n, _ptr(Q), m, _ptr(out), _ptr(gcd), _ptr(ghd),
                                 _ptr(ws), ws.numel(), _stream(P.device)), ctx.handle)
    cd, hd = out[:, 0], out[:, 1]
    if squeeze:
        return cd[0], hd[0], (None if gcd is None else gcd[0]), (None if ghd is None else ghd[0])
    return cd, hd, gcd, ghd


class ChamferFn(torch.autograd.Function):
    """CD(P, Q) as a differentiable loss in P (the target Q gets no gradient)."""

    @staticmethod
    def forward(fctx, P, Q, which):
        cd, hd, gcd, ghd = chamfer_hausdorff(P, Q, grads=True)
        fctx.save_for_backward(gcd if which == "chamfer" else ghd)
        return cd if which == "chamfer" else hd

    @staticmethod
    def backward(fctx, g):
        (gp,) = fctx.saved_tensors
        scale = g.reshape(g.shape + (1,) * (gp.dim() - g.dim()))
        return gp * scale, None, None


def chamfer_loss(P, Q):
    return ChamferFn.apply(P.contiguous(), Q.contiguous(), "chamfer")


def hausdorff_loss(P, Q):
    return ChamferFn.apply(P.contiguous(), Q.contiguous(), "hausdorff")


# --------------------------------------------------------------------------
# ragged batches
# --------------------------------------------------------------------------

class SurfaceBatch:
    """A ragged batch plan (nurbs_plan_*): surfaces of uneven degree, control
    grid and sample grid, one persistent launch per direction.

    ``shapes`` int [n][6] = (p, q, nu_c, nv_c, nu_s, nv_s); ``offsets`` int
    [n][7] element offsets of (ctrl, w, ku, kv, us, vs, pts) in the packed
    arrays passed to ``forward`` / ``backward``."""

    def __init__(self, shapes, offsets, device: int | None = None, validate: bool = False,
                 ctx: Context | None = None):
        shapes = np.ascontiguousarray(shapes, np.int64)
        offsets = np.ascontiguousarray(offsets, np.int64)
        n = int(shapes.shape[0])
        self.n = n
        self.ctx = ctx or context(device)
        self.device = torch.device("cuda", self.ctx.device)
        arr = (N.nurbs_desc * max(n, 1))()
        for s in range(n):
            d = arr[s]
            d.p, d.q, d.nu_c, d.nv_c, d.nu_s, d.nv_s = (int(x) for x in shapes[s])
            (d.ctrl_off, d.w_off, d.ku_off, d.kv_off, d.us_off, d.vs_off, d.pts_off) = (int(x) for x in offsets[s])
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        flags = N.NURBS_VALIDATE if validate else 0
        _check(N.lib().nurbs_plan_create(self.ctx.handle, arr, n, flags, ctypes.byref(h), ctypes.byref(ws)),
               self.ctx.handle)
        self.handle = h
        self.ws_bytes = ws.value
        self.validate = validate
        self.shapes, self.offsets = shapes, offsets
        s = shapes
        self.n_pts_floats = int((offsets[:, 6] + s[:, 4] * s[:, 5] * 3).max()) if n else 0
        self.n_points = int((s[:, 4] * s[:, 5]).sum()) if n else 0
        self._ws = None

    def info(self):
        f, b, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(N.lib().nurbs_plan_info(self.handle, ctypes.byref(f), ctypes.byref(b), ctypes.byref(g)))
        return {"fwd_tiles": f.value, "bwd_tiles": b.value, "grid": g.value}

    def workspace(self):
        """The plan's workspace (allocated once, reused by every call)."""
        if self._ws is None:
            self._ws = torch.zeros(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def forward(self, ctrl, w, ku, kv, us, vs, out=None, stream=None):
        if out is None:
            out = torch.empty(self.n_pts_floats, dtype=torch.float32, device=self.device)
        ws = self.workspace()
        st = stream.cuda_stream if stream is not None else _stream(self.device)
        _check(N.lib().nurbs_plan_fwd(self.handle, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv), _ptr(us), _ptr(vs),
                                      _ptr(out), _ptr(ws), ws.numel(), st), self.ctx.handle)
        return out

    def backward(self, ctrl, w, ku, kv, us, vs, grad_pts, mask: int = N.NURBS_GRAD_ALL, out=None, stream=None):
        if out is None:
            out = (torch.empty_like(ctrl) if mask & 1 else None, torch.empty_like(w) if mask & 2 else None,
                   torch.empty_like(ku) if mask & 4 else None, torch.empty_like(kv) if mask & 8 else None)
        gc, gw, gu, gv = out
        ws = self.workspace()
        st = stream.cuda_stream if stream is not None else _stream(self.device)
        _check(N.lib().nurbs_plan_bwd(self.handle, _ptr(ctrl), _ptr(w), _ptr(ku), _ptr(kv), _ptr(us), _ptr(vs),
                                      _ptr(grad_pts), _ptr(gc), _ptr(gw), _ptr(gu), _ptr(gv), int(mask), _ptr(ws),
                                      ws.numel(), st), self.ctx.handle)
        return out

    def set_timing(self, max_calls: int):
        """Record HIP events around this plan's kernels (0 turns it off)."""
        _check(N.lib().nurbs_plan_set_timing(self.handle, int(max_calls)), self.ctx.handle)
        self._timing_slots = int(max_calls)

    def read_timing(self):
        """Per recorded call: forward, backward row-loop, gather and finalize kernel ms."""
        n = max(getattr(self, "_timing_slots", 0), 1)
        f = (ctypes.c_float * n)()
        b = (ctypes.c_float * n)()
        g = (ctypes.c_float * n)()
        z = (ctypes.c_float * n)()
        nf, nb = ctypes.c_int(), ctypes.c_int()
        _check(N.lib().nurbs_plan_read_timing(self.handle, f, ctypes.byref(nf), b, g, z, ctypes.byref(nb)),
               self.ctx.handle)
        return (np.array(f[:nf.value]), np.array(b[:nb.value]), np.array(g[:nb.value]), np.array(z[:nb.value]))

    def read_device_error(self, stream=None) -> int:
        code = ctypes.c_int()
        st = stream.cuda_stream if stream is not None else _stream(self.device)
        _check(N.lib().nurbs_read_device_error(_ptr(self.workspace()), st, ctypes.byref(code)))
        return code.value

    def close(self):
        if getattr(self, "handle", None):
            N.lib().nurbs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# test exports
# --------------------------------------------------------------------------

def find_spans(knots, p: int, x):
    _need_cuda_f32("knots", knots)
    _need_cuda_f32("x", x)
    out = torch.empty(x.numel(), dtype=torch.int32, device=x.device)
    _check(N.lib().nurbs_find_spans(_ptr(knots), knots.numel(), int(p), _ptr(x), x.numel(), _ptr(out),
                                    _stream(x.device)))
    return out


def basis(knots, p: int, x):
    _need_cuda_f32("knots", knots)
    _need_cuda_f32("x", x)
    out = torch.empty((x.numel(), p + 1), dtype=torch.float32, device=x.device)
    _check(N.lib().nurbs_basis(_ptr(knots), knots.numel(), int(p), _ptr(x), x.numel(), _ptr(out),
                               _stream(x.device)))
    return out


# --------------------------------------------------------------------------
# tile autotuning
# --------------------------------------------------------------------------

TILE_CANDIDATES = (2048, 4096, 8192, 16384, 65536)
SCHEDULES = (N.NURBS_SCHED_DYNAMIC, N.NURBS_SCHED_STATIC)


def autotune(shapes, offsets, inputs, upstream, device: int | None = None, candidates=TILE_CANDIDATES,
             schedules=SCHEDULES, reps: int = 5, validate: bool = False):
    """Pick the tile schedule and the forward and backward tile sizes for a
    ragged batch by timing.

    Every (schedule, target sample points per tile) pair is timed on the
    batch itself -- the forward and the backward (with its finalize)
    separately, ``reps`` calls each after a warm-up call, with HIP events on
    the plan's stream -- and the fastest of each direction is kept (the
    schedule by the sum of the two).  Returns ``(plan, report)``: a
    SurfaceBatch built with the chosen settings (on a context of its own)
    and the timings in ms per candidate, keyed "<schedule>:<points>"."""
    ctrl, w, ku, kv, us, vs = inputs
    dev = ctrl.device
    report = {"fwd": {}, "bwd": {}}
    pts = None
    grads = (torch.empty_like(ctrl), torch.empty_like(w), torch.empty_like(ku), torch.empty_like(kv))
    names = {N.NURBS_SCHED_DYNAMIC: "dynamic", N.NURBS_SCHED_STATIC: "static"}
    for sched in schedules:
      for cand in candidates:
        ctx = Context(device, validate=validate)
        ctx.set_tiling(cand, cand)
        ctx.set_schedule(sched)
        plan = SurfaceBatch(shapes, offsets, device=device, validate=validate, ctx=ctx)
        if pts is None:
            pts = torch.empty(plan.n_pts_floats, dtype=torch.float32, device=dev)
        plan.workspace()
        plan.forward(ctrl, w, ku, kv, us, vs, out=pts)
        plan.backward(ctrl, w, ku, kv, us, vs, upstream, out=grads)
        torch.cuda.synchronize(dev)
        plan.set_timing(reps)
        for _ in range(reps):
            plan.forward(ctrl, w, ku, kv, us, vs, out=pts)
            plan.backward(ctrl, w, ku, kv, us, vs, upstream, out=grads)
        torch.cuda.synchronize(dev)
        f, b, g, z = plan.read_timing()
        plan.set_timing(0)
        key = f"{names[sched]}:{cand}"
        report["fwd"][key] = float(np.median(f))
        report["bwd"][key] = float(np.median(b + g + z))
        plan.close()
        del plan
    # one schedule for both directions (a plan has one), then the best tiling of each
    best_sched = min(schedules, key=lambda sc: min(v for k, v in report["fwd"].items() if k.startswith(names[sc]))
                     + min(v for k, v in report["bwd"].items() if k.startswith(names[sc])))
    pref = names[best_sched] + ":"
    best_f = int(min((k for k in report["fwd"] if k.startswith(pref)), key=report["fwd"].get).split(":")[1])
    best_b = int(min((k for k in report["bwd"] if k.startswith(pref)), key=report["bwd"].get).split(":")[1])
    ctx = Context(device, validate=validate)
    ctx.set_tiling(best_f, best_b)
    ctx.set_schedule(best_sched)
    report["chosen"] = {"schedule": names[best_sched], "fwd_tile_points": best_f, "bwd_tile_points": best_b}
    return SurfaceBatch(shapes, offsets, device=device, validate=validate, ctx=ctx), report
