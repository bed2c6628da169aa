"""Surface fitting with the library's forward and adjoint (Sec. 4.2 of
NURBS-Diff: fit a NURBS surface to sampled points by gradient descent on the
control points, weights and knots).

One step: S = surface(P, W, U, V) on the sample grid (library forward),
g = dL/dS = 2 (S - T) for L = sum ||S - T||^2, the library's backward for
dL/dP, dL/dW, dL/dU, dL/dV, an Adam update, then the projections that keep
the surface valid: weights at least ``w_min``, the clamped end knots fixed,
and the interior knots kept in order inside [0, 1] with gaps of at least
``knot_gap`` (so no span collapses and the knot derivative, which scales
with the inverse square of a span, stays finite).  The projection is a
running maximum and a running minimum, so each knot keeps its index and its
Adam moments.

With fixed knots (``train_knots=False``) the spans and basis values of the
sample grid are computed once into tables (the fixed-knot B-spline layer
with a precomputed basis) and every step reads them
(``nurbs_surface_fwd_tab`` / ``nurbs_surface_bwd_tab``) unless
``cached_basis=False``.

The fit owns a library context whose tiling (sample points per forward and
backward tile) is chosen at construction by timing the candidates on the
problem itself (``tiling="auto"``): one surface of 512 x 512 samples makes
only 16 tiles at the default 16384 points per tile, far too few waves for
the chip.  The summation order, and so the bits of the result, depend on
the tiling only.

With ``graph=True`` the whole step (both library launches, the loss gradient,
Adam and the projections) is captured once in a HIP graph and replayed, so a
step costs one graph launch.  Every buffer is allocated before capture.
"""
from __future__ import annotations

import torch

from . import _native as N
from .api import Context, basis_table, surface_bwd, surface_bwd_tab, surface_fwd, surface_fwd_tab

# points per tile tried by the tiling search: a single surface needs small
# tiles to occupy the chip, a large one amortises the per-tile set-up
FIT_TILE_CANDIDATES = (256, 512, 1024, 2048, 4096, 16384)


def project_knots(inner, ramp, top: float):
    """In place: the closest-from-below ordering of the interior knots x_1..x_n
    with x_1 >= g, x_{i+1} >= x_i + g and x_n <= 1 - g (ramp = i * g,
    top = 1 - (n + 1) g): a running maximum of x_i - i g (floored at 0)
    pushes knots up, then a running minimum from the right caps them."""
    lo = torch.cummax(torch.clamp(inner - ramp, min=0.0), 0).values
    hi = torch.flip(torch.cummin(torch.flip(torch.clamp(lo, max=top), [0]), 0).values, [0])
    inner.copy_(hi + ramp)


class SurfaceFit:
    """Fit one surface of degree (p, q) to a target grid.

    ctrl [nu_c, nv_c, 3], w [nu_c, nv_c], ku [nu_c + p + 1], kv [nv_c + q + 1],
    us [nu_s], vs [nv_s], target [nu_s, nv_s, 3]: float32 CUDA tensors (copied).
    """

    def __init__(self, ctrl, w, ku, kv, p: int, q: int, us, vs, target, lr: float = 1e-2,
                 train_knots: bool = True, w_min: float = 1e-3, knot_gap: float = 1e-3, graph: bool = True,
                 cached_basis: bool = True, tiling="auto"):
        self.p, self.q = int(p), int(q)
        self.ctrl = ctrl.detach().clone().contiguous()
        self.w = w.detach().clone().contiguous()
        self.ku = ku.detach().clone().contiguous()
        self.kv = kv.detach().clone().contiguous()
        self.us, self.vs = us.contiguous(), vs.contiguous()
        self.target = target.contiguous()
        self.train_knots = bool(train_knots)
        self.w_min = float(w_min)
        self.nu_c, self.nv_c = int(ctrl.shape[0]), int(ctrl.shape[1])
        # ramps i * gap (i = 1..n) of the knot projection, one per direction
        self.ramps = []
        for d, nc in ((self.p, self.nu_c), (self.q, self.nv_c)):
            n = nc - d - 1
            gap = min(float(knot_gap), 0.5 / (n + 1)) if n > 0 else 0.0
            r = torch.arange(1, n + 1, dtype=torch.float32, device=ctrl.device) * gap
            self.ramps.append((r, 1.0 - (n + 1) * gap))
        self.mask = N.NURBS_GRAD_CTRL | N.NURBS_GRAD_W
        params = [self.ctrl, self.w]
        if self.train_knots:
            self.mask |= N.NURBS_GRAD_KU | N.NURBS_GRAD_KV
            params += [self.ku, self.kv]
        self.params = params
        # fixed knots: spans and basis of the sample grid, computed once
        self.tabs = None
        if not self.train_knots and cached_basis:
            self.tabs = (basis_table(self.ku, self.p, self.us), basis_table(self.kv, self.q, self.vs))
        self.pts = torch.empty_like(self.target)
        self.g = torch.empty_like(self.target)
        self.ctx = Context(ctrl.device.index)
        if tiling == "auto":
            tiling = self._tune_tiling()
        if tiling:
            self.ctx.set_tiling(*tiling)
        self.tiling = getattr(self.ctx, "tiling", (16384, 16384))
        for t in params:
            t.grad = torch.zeros_like(t)
        # capturable in both modes, so eager and graph steps run the same arithmetic
        self.opt = torch.optim.Adam(params, lr=lr, capturable=True)
        self.graph = None
        self.steps = 0
        if graph:
            self._capture()

    def _fwd(self):
        if self.tabs is not None:
            tu, tv = self.tabs
            surface_fwd_tab(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs, tu, tv,
                            out=self.pts, ctx=self.ctx)
        else:
            surface_fwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs, out=self.pts,
                        ctx=self.ctx)

    def _bwd(self):
        if self.tabs is not None:
            gc, gw = surface_bwd_tab(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs,
                                     *self.tabs, self.g, mask=self.mask, ctx=self.ctx)
            return gc, gw, None, None
        return surface_bwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs, self.g,
                           mask=self.mask, ctx=self.ctx)

    def _tune_tiling(self, reps: int = 5):
        """The forward and the backward tile sizes that run fastest on this
        problem (HIP events around each call, median of ``reps``)."""
        self.g.zero_()
        best = {}
        for cand in FIT_TILE_CANDIDATES:
            self.ctx.set_tiling(cand, cand)
            self._fwd()
            self._bwd()
            times = {"fwd": [], "bwd": []}
            for _ in range(reps):
                for k, fn in (("fwd", self._fwd), ("bwd", self._bwd)):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    fn()
                    b.record()
                    times[k].append((a, b))
            torch.cuda.synchronize()
            for k, ev in times.items():
                t = sorted(x.elapsed_time(y) for x, y in ev)[len(ev) // 2]
                if k not in best or t < best[k][0]:
                    best[k] = (t, cand)
        return best["fwd"][1], best["bwd"][1]

    # -- one step, written with preallocated tensors only ------------------
    def _step_body(self):
        self._fwd()
        torch.sub(self.pts, self.target, out=self.g)
        self.g.mul_(2.0)
        gc, gw, gu, gv = self._bwd()
        self.ctrl.grad.copy_(gc)
        self.w.grad.copy_(gw)
        if self.train_knots:
            # the clamped end knots stay fixed
            gu[: self.p + 1].zero_()
            gu[self.nu_c:].zero_()
            gv[: self.q + 1].zero_()
            gv[self.nv_c:].zero_()
            self.ku.grad.copy_(gu)
            self.kv.grad.copy_(gv)
        self.opt.step()
        with torch.no_grad():
            self.w.clamp_(min=self.w_min)
            if self.train_knots:
                for U, d, nc, (ramp, top) in ((self.ku, self.p, self.nu_c, self.ramps[0]),
                                              (self.kv, self.q, self.nv_c, self.ramps[1])):
                    if nc - d - 1 > 0:
                        project_knots(U[d + 1:nc], ramp, top)

    def _capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        saved = [t.detach().clone() for t in self.params]
        with torch.cuda.stream(side):
            for _ in range(3):  # warm-up: optimizer state and library contexts exist before capture
                self._step_body()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        # undo the warm-up steps: parameters and optimizer state back to the start
        with torch.no_grad():
            for t, s in zip(self.params, saved):
                t.copy_(s)
            for st in self.opt.state.values():
                for k, v in st.items():
                    if torch.is_tensor(v):
                        v.zero_()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_body()
        torch.cuda.synchronize()

    def step(self, n: int = 1):
        for _ in range(n):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._step_body()
        self.steps += n

    @torch.no_grad()
    def loss(self) -> float:
        """L = sum ||S - T||^2 at the current parameters (evaluated eagerly)."""
        S = surface_fwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs, ctx=self.ctx)
        return float(((S.double() - self.target.double()) ** 2).sum())
