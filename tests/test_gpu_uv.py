"""GPU parity of the scattered-pair calls (nurbs_surface_uv_fwd /
nurbs_surface_uv_bwd) against the oracle's scattered functions, through the
C ABI.

Bars: points within 1e-5 of the bounding-box diagonal of the oracle's
points, per surface; dS/du, dS/dv within 1e-5 of their largest magnitude;
gradients within 1e-4 of each tensor's largest magnitude, per surface, both
sides fed the same float32 dL/dS.  Cases: degree pairs from (1,1) to (7,7)
and unequal ones, the LDS and the global accumulator paths (small and
48x48 nets), pairs on (repeated) knots and outside the domain, shared and
per-surface pairs, no pairs, bitwise repeats, the grid of all pairs against
the grid calls, autograd and NURBS_VALIDATE.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_14547_amd as nd  # noqa: E402
from paper_2104_14547_amd import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def H(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_case(ub, derivs=True):
    ctrl, w, ku, kv, uv = T(ub.ctrl), T(ub.w), T(ub.ku), T(ub.kv), T(ub.uv)
    p, q = ub.p, ub.q
    if derivs:
        pts, du, dv = nd.api.surface_uv_fwd(ctrl, w, ku, kv, p, q, uv, derivs=True)
    else:
        pts = nd.api.surface_uv_fwd(ctrl, w, ku, kv, p, q, uv)
    grads = nd.api.surface_uv_bwd(ctrl, w, ku, kv, p, q, uv, T(ub.upstream))
    torch.cuda.synchronize()
    for b in range(ub.B):
        uvb = ub.uv if ub.uv.ndim == 2 else ub.uv[b]
        if ub.npts:
            S, Su, Sv = O.scattered_fwd(ub.ctrl[b], ub.w[b], ub.ku[b], ub.kv[b], p, q, uvb, derivs=True)
            diag = np.linalg.norm(S.max(0) - S.min(0))
            if diag == 0:
                c = ub.ctrl[b].reshape(-1, 3)
                diag = np.linalg.norm(c.max(0) - c.min(0))
            err = np.linalg.norm(H(pts[b]) - S, axis=1).max() / diag
            assert err <= 1e-5, f"surface {b}: point error {err:.3e}"
            if derivs:
                for got, want, nm in ((du, Su, "du"), (dv, Sv, "dv")):
                    e = np.abs(H(got[b]) - want).max() / np.abs(want).max()
                    assert e <= 1e-5, f"surface {b}: {nm} error {e:.3e}"
        ref = O.scattered_bwd(ub.ctrl[b], ub.w[b], ub.ku[b], ub.kv[b], p, q, uvb,
                              ub.upstream[b].astype(np.float64))
        for nm, got, want in zip(("ctrl", "w", "ku", "kv"), grads, ref):
            g = H(got[b]).ravel()
            r = want.ravel()
            sc = np.abs(r).max()
            e = np.abs(g - r).max() / sc if sc > 0 else np.abs(g).max()
            assert e <= 1e-4, f"surface {b} grad {nm}: rel err {e:.3e}"
    return pts, grads


@pytest.mark.parametrize("p,q", [(1, 1), (2, 3), (3, 3), (3, 1), (4, 5), (5, 5), (7, 6), (7, 7)])
def test_uv_parity_degrees(p, q):
    ub = W.uv_batch(seed=10 * p + q, B=3, p=p, q=q, nu_c=max(p + 1, 11), nv_c=max(q + 1, 9), npts=2000,
                    repeat=0.15)
    run_case(ub)


def test_uv_global_accumulator_path():
    # 48x48 net: 4*2304 + 52 + 52 accumulators exceed the LDS copy
    ub = W.uv_batch(seed=3, B=2, p=3, q=2, nu_c=48, nv_c=48, npts=6000)
    run_case(ub, derivs=False)


def test_uv_shared_pairs_large_batch():
    ub = W.uv_batch(seed=4, B=24, p=3, q=3, nu_c=12, nv_c=14, npts=700, shared_uv=True)
    run_case(ub, derivs=False)


def test_uv_on_knots_and_outside():
    ub = W.uv_batch(seed=5, B=2, p=3, q=2, nu_c=9, nv_c=8, npts=64, repeat=0.5)
    ub.ku[:] = ub.ku[0]
    ub.kv[:] = ub.kv[0]
    us = np.concatenate([ub.ku[0], [-0.3, 1.2]])
    vs = np.concatenate([ub.kv[0], [1.5, -0.1]])
    g = np.random.Generator(np.random.PCG64(1))
    pairs = np.stack([g.choice(us, 64), g.choice(vs, 64)], -1).astype(np.float32)
    ub.uv = np.stack([pairs, pairs[::-1]])
    run_case(ub)


def test_uv_grid_of_all_pairs_matches_grid_call():
    b = W.batch_bicubic(1, n_surf=2, nc=10, ns=24)
    s = b.surface(1)
    uu, vv = np.meshgrid(s["us"], s["vs"], indexing="ij")
    uv = np.stack([uu.ravel(), vv.ravel()], -1).astype(np.float32)
    perm = np.random.Generator(np.random.PCG64(2)).permutation(len(uv))
    ctrl, w, ku, kv = T(s["ctrl"]), T(s["w"]), T(s["ku"]), T(s["kv"])
    grid = nd.api.surface_fwd(ctrl, w, ku, kv, 3, 3, T(s["us"]), T(s["vs"])).reshape(-1, 3)
    sc = nd.api.surface_uv_fwd(ctrl, w, ku, kv, 3, 3, T(uv[perm]))
    diag = float((grid.max(0).values - grid.min(0).values).norm())
    assert float((sc - grid[perm]).norm(dim=1).max()) <= 1e-5 * diag


def test_uv_empty_repeat_autograd_validate():
    ub = W.uv_batch(seed=6, B=2, p=2, q=3, nu_c=7, nv_c=8, npts=0)
    ctrl, w, ku, kv, uv = T(ub.ctrl), T(ub.w), T(ub.ku), T(ub.kv), T(ub.uv)
    gs = nd.api.surface_uv_bwd(ctrl, w, ku, kv, 2, 3, uv, torch.zeros((2, 0, 3), device="cuda"))
    assert all(float(g.abs().sum()) == 0.0 for g in gs)
    ub = W.uv_batch(seed=7, B=2, p=3, q=3, nu_c=20, nv_c=20, npts=5000)
    ctrl, w, ku, kv, uv, g = T(ub.ctrl), T(ub.w), T(ub.ku), T(ub.kv), T(ub.uv), T(ub.upstream)
    a = nd.api.surface_uv_bwd(ctrl, w, ku, kv, 3, 3, uv, g)
    b = nd.api.surface_uv_bwd(ctrl, w, ku, kv, 3, 3, uv, g)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for t in (ctrl, w, ku, kv):
        t.requires_grad_(True)
    (nd.api.surface_uv(ctrl, w, ku, kv, 3, 3, uv) * g).sum().backward()
    for t, x in zip((ctrl, w, ku, kv), a):
        assert torch.equal(t.grad, x)
    ctx = nd.api.Context(0, validate=True)
    bad = uv.detach().clone()
    bad[0, 5, 0] = 2.0
    nd.api.surface_uv_fwd(ctrl.detach(), w.detach(), ku.detach(), kv.detach(), 3, 3, bad, ctx=ctx)
    assert ctx.read_device_error(ctx.last_ws) == nd.api.N.NURBS_EDOMAIN
