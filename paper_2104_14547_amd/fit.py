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

With ``graph=True`` the whole step (both library launches, the loss gradient,
Adam and the projections) is captured once in a HIP graph and replayed, so a
step costs one graph launch.  Every buffer is allocated before capture.
"""
from __future__ import annotations

import torch

from . import _native as N
from .api import surface_bwd, surface_fwd


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
                 train_knots: bool = True, w_min: float = 1e-3, knot_gap: float = 1e-3, graph: bool = True):
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
        self.pts = torch.empty_like(self.target)
        self.g = torch.empty_like(self.target)
        for t in params:
            t.grad = torch.zeros_like(t)
        # capturable in both modes, so eager and graph steps run the same arithmetic
        self.opt = torch.optim.Adam(params, lr=lr, capturable=True)
        self.graph = None
        self.steps = 0
        if graph:
            self._capture()

    # -- one step, written with preallocated tensors only ------------------
    def _step_body(self):
        surface_fwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs, out=self.pts)
        torch.sub(self.pts, self.target, out=self.g)
        self.g.mul_(2.0)
        gc, gw, gu, gv = surface_bwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs,
                                     self.g, mask=self.mask)
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
        S = surface_fwd(self.ctrl, self.w, self.ku, self.kv, self.p, self.q, self.us, self.vs)
        return float(((S.double() - self.target.double()) ** 2).sum())
