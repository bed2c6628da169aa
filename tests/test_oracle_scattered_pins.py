"""Pins for the oracle's scattered-parameter surface functions (eq. NURBS at
each (u, v) pair).

* The pairs of a tensor-product grid, given in a shuffled order, reproduce
  the grid oracle's points point for point and its gradients (sums over the
  same terms in another order) to 1e-12 relative -- the grid oracle is
  pinned independently (test_oracle_pins).
* Central finite differences of L = sum g . S in P, w and interior knots on
  scattered pairs, including pairs outside the domain (clamped, no
  parameter gradient) and pairs on knots.
* S_u, S_v by finite differences in the parameters.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_14547_amd import workloads as W


def surf(seed, p, q, nu_c, nv_c):
    g = np.random.default_rng(seed)
    ctrl = W.perturbed_lattice(g, nu_c, nv_c).astype(np.float64)
    w = g.uniform(0.5, 1.5, (nu_c, nv_c))
    ku = W.clamped_random_knots(g, nu_c, p, 0.2).astype(np.float64)
    kv = W.clamped_random_knots(g, nv_c, q, 0.2).astype(np.float64)
    return g, ctrl, w, ku, kv


@pytest.mark.parametrize("p,q", [(1, 2), (3, 3), (2, 5)])
def test_shuffled_grid_equals_grid(p, q):
    g, ctrl, w, ku, kv = surf(p * 10 + q, p, q, 9, 7)
    us = np.concatenate([W.uniform_grid(11), ku[p + 1:p + 3]]).astype(np.float64)
    vs = W.uniform_grid(13).astype(np.float64)
    us.sort()
    S = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs)
    G = g.uniform(-1, 1, S.shape)
    want = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G)
    uu, vv = np.meshgrid(us, vs, indexing="ij")
    uv = np.stack([uu.ravel(), vv.ravel()], 1)
    perm = g.permutation(len(uv))
    Ss = O.scattered_fwd(ctrl, w, ku, kv, p, q, uv[perm])
    np.testing.assert_array_equal(Ss, S.reshape(-1, 3)[perm])
    got = O.scattered_bwd(ctrl, w, ku, kv, p, q, uv[perm], G.reshape(-1, 3)[perm])
    for a, b in zip(got, want):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


def test_scattered_finite_differences():
    p, q = 3, 2
    g, ctrl, w, ku, kv = surf(5, p, q, 7, 6)
    uv = np.concatenate([g.uniform(-0.05, 1.05, (40, 2)), [[ku[4], 0.3], [0.5, kv[3]], [1.0, 1.0]]])
    G = g.uniform(-1, 1, (len(uv), 3))
    dP, dW, dU, dV = O.scattered_bwd(ctrl, w, ku, kv, p, q, uv, G)
    L = lambda c, ww, a, b: float((O.scattered_fwd(c, ww, a, b, p, q, uv) * G).sum())
    h = 1e-6
    for (i, j, x) in [(0, 0, 0), (3, 2, 1), (6, 5, 2), (2, 4, 0)]:
        cp, cm = ctrl.copy(), ctrl.copy()
        cp[i, j, x] += h
        cm[i, j, x] -= h
        assert (L(cp, w, ku, kv) - L(cm, w, ku, kv)) / (2 * h) == pytest.approx(dP[i, j, x], rel=1e-6, abs=1e-8)
        wp, wm = w.copy(), w.copy()
        wp[i, j] += h
        wm[i, j] -= h
        assert (L(ctrl, wp, ku, kv) - L(ctrl, wm, ku, kv)) / (2 * h) == pytest.approx(dW[i, j], rel=1e-6, abs=1e-8)
    # interior simple knots with no parameter nearby
    for k in range(p + 1, len(ku) - p - 1):
        if ku[k] in (ku[k - 1], ku[k + 1]) or np.abs(uv[:, 0] - ku[k]).min() < 1e-4:
            continue
        a, b = ku.copy(), ku.copy()
        a[k] += h
        b[k] -= h
        assert (L(ctrl, w, a, kv) - L(ctrl, w, b, kv)) / (2 * h) == pytest.approx(dU[k], rel=1e-5, abs=1e-7)
    for k in range(q + 1, len(kv) - q - 1):
        if kv[k] in (kv[k - 1], kv[k + 1]) or np.abs(uv[:, 1] - kv[k]).min() < 1e-4:
            continue
        a, b = kv.copy(), kv.copy()
        a[k] += h
        b[k] -= h
        assert (L(ctrl, w, ku, a) - L(ctrl, w, ku, b)) / (2 * h) == pytest.approx(dV[k], rel=1e-5, abs=1e-7)


def test_scattered_parametric_derivatives():
    p, q = 2, 3
    g, ctrl, w, ku, kv = surf(6, p, q, 6, 8)
    uv = g.uniform(0.02, 0.98, (30, 2))
    S, Su, Sv = O.scattered_fwd(ctrl, w, ku, kv, p, q, uv, derivs=True)
    h = 1e-7
    for col, D in ((0, Su), (1, Sv)):
        a, b = uv.copy(), uv.copy()
        a[:, col] += h
        b[:, col] -= h
        fd = (O.scattered_fwd(ctrl, w, ku, kv, p, q, a) - O.scattered_fwd(ctrl, w, ku, kv, p, q, b)) / (2 * h)
        # one-sided at knots: skip pairs within h of a knot
        knots = ku if col == 0 else kv
        ok = np.abs(uv[:, col][:, None] - knots[None, :]).min(1) > 1e-5
        np.testing.assert_allclose(fd[ok], D[ok], rtol=1e-5, atol=1e-6)
