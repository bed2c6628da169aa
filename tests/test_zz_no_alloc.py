"""nurbs_surface_bwd_noalloc (the backward for callers that cannot allocate)
against nurbs_surface_bwd, through the C ABI.

Two calls in a row on the device's one scratch array, the second with a
smaller input, each compared with nurbs_surface_bwd given a caller
workspace: the two share their kernels and tiling, so the gradients must be
equal bit for bit, and both are checked against the FP64 oracle at the
parity bar (gradients within 1e-4 of each tensor's largest magnitude).  Also:
a shape whose slots exceed the 64 MiB scratch is refused with
NURBS_EWORKSPACE before anything runs, and NURBS_VALIDATE is refused.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_14547_amd as nd  # noqa: E402
from paper_2104_14547_amd import _native as N  # noqa: E402
from paper_2104_14547_amd import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def uniform_inputs(batch):
    """Dense [B, ...] tensors of a packed batch whose surfaces share one shape."""
    B = batch.n
    p, q, nu_c, nv_c, nu_s, nv_s = (int(x) for x in batch.shapes[0])
    assert (batch.shapes == batch.shapes[0]).all()
    ctrl = T(batch.ctrl.reshape(B, nu_c, nv_c, 3))
    w = T(batch.w.reshape(B, nu_c, nv_c))
    ku = T(batch.ku.reshape(B, nu_c + p + 1))
    kv = T(batch.kv.reshape(B, nv_c + q + 1))
    us = T(batch.us.reshape(B, nu_s))
    vs = T(batch.vs.reshape(B, nv_s))
    g = T(batch.upstream.reshape(B, nu_s, nv_s, 3))
    return (p, q, nu_c, nv_c, nu_s, nv_s), (ctrl, w, ku, kv, us, vs), g


def call_noalloc(ctx, shape, x, g):
    p, q, nu_c, nv_c, nu_s, nv_s = shape
    ctrl, w, ku, kv, us, vs = x
    B = ctrl.shape[0]
    out = (torch.full_like(ctrl, float("nan")), torch.full_like(w, float("nan")),
           torch.full_like(ku, float("nan")), torch.full_like(kv, float("nan")))
    rc = N.lib().nurbs_surface_bwd_noalloc(
        ctx.handle, B, p, q, nu_c, nv_c, ctrl.data_ptr(), w.data_ptr(), ku.data_ptr(), kv.data_ptr(), nu_s, nv_s,
        us.data_ptr(), vs.data_ptr(), 0, g.data_ptr(), *[t.data_ptr() for t in out], N.NURBS_GRAD_ALL,
        torch.cuda.current_stream().cuda_stream)
    assert rc == 0, N.lib().nurbs_last_error(ctx.handle).decode()
    return out


def with_upstream(batch, seed):
    batch.upstream = np.random.Generator(np.random.PCG64(seed)).uniform(
        -0.1, 0.1, batch.n_pts_floats).astype(np.float32)
    return batch


def small_batch():
    g = np.random.Generator(np.random.PCG64(77))
    parts = []
    for _ in range(8):
        p, q, nu_c, nv_c, nu_s, nv_s = 2, 4, 10, 13, 50, 70
        parts.append(dict(p=p, q=q, nu_c=nu_c, nv_c=nv_c, nu_s=nu_s, nv_s=nv_s,
                          ctrl=W.perturbed_lattice(g, nu_c, nv_c), w=g.uniform(0.5, 1.5, (nu_c, nv_c)),
                          ku=W.clamped_random_knots(g, nu_c, p, 0.2), kv=W.clamped_random_knots(g, nv_c, q, 0.2),
                          us=W.uniform_grid(nu_s), vs=W.uniform_grid(nv_s)))
    return with_upstream(W.pack("noalloc_small", parts), 78)


def check_against_oracle(batch, grads):
    want = O.bwd(batch, batch.upstream.astype(np.float64))
    for name, got, ref in zip(("ctrl", "w", "ku", "kv"), grads, want):
        got = got.detach().cpu().numpy().reshape(batch.n, -1).astype(np.float64)
        ref = ref.reshape(batch.n, -1)
        for s in range(batch.n):
            scale = np.abs(ref[s]).max()
            err = np.abs(got[s] - ref[s]).max() / scale
            assert err <= GRAD_TOL, f"surface {s} grad {name}: rel err {err:.3e}"


def test_noalloc_matches_workspace_backward_twice():
    ctx = nd.api.Context(0)
    for batch in (with_upstream(W.batch_bicubic(1), 9), small_batch()):
        shape, x, g = uniform_inputs(batch)
        got = call_noalloc(ctx, shape, x, g)
        ref = nd.api.surface_bwd(*x[:4], shape[0], shape[1], *x[4:], g, ctx=ctx)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        check_against_oracle(batch, got)


def test_noalloc_refuses_oversized_and_validate():
    ctx = nd.api.Context(0)
    rc = N.lib().nurbs_surface_bwd_noalloc(ctx.handle, 4096, 3, 3, 48, 48, None, None, None, None, 256, 256, None,
                                           None, 1, None, None, None, None, None, N.NURBS_GRAD_ALL, None)
    assert rc == N.NURBS_EWORKSPACE
    assert "scratch" in N.lib().nurbs_last_error(ctx.handle).decode()
    need = ctypes.c_size_t()
    assert N.lib().nurbs_surface_ws_bytes(ctx.handle, 4096, 3, 3, 48, 48, 256, 256, N.NURBS_GRAD_ALL,
                                          ctypes.byref(need)) == 0
    assert need.value > 64 << 20
    vctx = nd.api.Context(0, validate=True)
    rc = N.lib().nurbs_surface_bwd_noalloc(vctx.handle, 1, 3, 3, 8, 8, None, None, None, None, 16, 16, None,
                                           None, 1, None, None, None, None, None, N.NURBS_GRAD_ALL, None)
    assert rc == N.NURBS_EUNSUPPORTED
