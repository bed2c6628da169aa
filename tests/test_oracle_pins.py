"""Pins for the FP64 oracle, against facts the paper and mathematics fix.

The paper prints no worked numeric example, so every pin here is a closed
form, an independent algorithm from the literature, an invariant of the
definitions, or a finite difference:

* knot span -- hand-derived cases of the half-open span rule (Sec. 3.1.2
  step 1) with the last-span reading at u = U_{n+1};
* basis -- partition of unity, non-negativity, local support, the Bernstein
  closed form on [0^{p+1}, 1^{p+1}], the uniform quadratic / cubic B-spline
  pieces, continuity at simple knots (eqs. NURBSBasis, BSplineBasis2);
* forward -- de Boor's corner-cutting algorithm on homogeneous points
  (an independent evaluator), the exact rational quarter circle, endpoint
  interpolation, weight-scale (projective) and affine invariance, the
  convex hull (eq. NURBS, Sec. 3.1.2 step 3);
* dS/du -- central differences of the forward (Appendix A);
* gradients -- central differences of the forward for P, W, U, V;
  translation invariance of dP, the zero weighted sum of dW, shift and
  scale invariance of dU/dV, the Bezier closed form for end-knot gradients
  (eqs. NURBSuDerivative4, NURBSvDerivative5, NURBSvDerivative6 and the
  knot recursion of Sec. 3.2.1);
* dense mode == local mode.
"""
import bisect
import math

import numpy as np
import pytest

from oracle import oracle as O


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rand_knots(g, n_ctrl, p, repeat=0.0):
    inner = np.sort(g.uniform(0.05, 0.95, n_ctrl - p - 1))
    if repeat > 0 and len(inner) > 1:
        m = 1
        for t in range(1, len(inner)):
            if g.uniform() < repeat and m < p:
                inner[t] = inner[t - 1]
                m += 1
            else:
                m = 1
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def rand_surface(g, p, q, nu_c, nv_c, repeat=0.0):
    ctrl = g.uniform(-1, 1, (nu_c, nv_c, 3))
    w = g.uniform(0.5, 1.5, (nu_c, nv_c))
    return ctrl, w, rand_knots(g, nu_c, p, repeat), rand_knots(g, nv_c, q, repeat)


# --------------------------------------------------------------------------
# knot span
# --------------------------------------------------------------------------

SPAN_CASES = [
    # (knots, p, u, span) -- half-open [U_k, U_{k+1}); u = U_{n+1} -> n;
    # parameters outside [U_p, U_{n+1}] are clamped first.
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 0.0, 3),
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 0.1, 3),
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 0.2, 4),   # on a knot: right interval
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 0.8, 7),
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 0.99, 7),
    ([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], 3, 1.0, 7),   # right end -> last span n
    ([0, 0, 0, .5, .5, 1, 1, 1], 2, 0.49, 2),
    ([0, 0, 0, .5, .5, 1, 1, 1], 2, 0.5, 4),                 # repeated knot: last copy
    ([0, 0, 0, .5, .5, 1, 1, 1], 2, 1.0, 4),
    ([0, 0, 0, .5, .5, 1, 1, 1], 2, -0.25, 2),               # clamped up to U_p
    ([0, 0, 0, .5, .5, 1, 1, 1], 2, 1.5, 4),                 # clamped down to U_{n+1}
    ([0, 1, 2, 3, 4, 5], 2, 2.0, 2),                          # unclamped: domain [U_2, U_3]
    ([0, 1, 2, 3, 4, 5], 2, 3.0, 2),
]


@pytest.mark.parametrize("U,p,u,k", SPAN_CASES)
def test_span_cases(U, p, u, k):
    assert O.find_span(np.array(U, float), p, u) == k


def test_span_matches_bisect_random():
    g = rng(11)
    for _ in range(200):
        p = int(g.integers(1, 6))
        U = rand_knots(g, int(g.integers(p + 1, 20)), p, repeat=0.3)
        n = len(U) - p - 2
        for u in np.concatenate([g.uniform(0, 1, 20), U]):
            k = min(max(bisect.bisect_right(list(U), u) - 1, p), n)
            assert O.find_span(U, p, u) == k


# --------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------

def test_partition_of_unity_nonneg_local_support():
    g = rng(12)
    for _ in range(100):
        p = int(g.integers(1, 8))
        U = rand_knots(g, int(g.integers(p + 1, 16)), p, repeat=0.3)
        for u in np.concatenate([g.uniform(0, 1, 10), [0.0, 1.0], U[p:len(U) - p]]):
            N, _, _ = O.basis_dense(U, p, u)
            assert abs(N.sum() - 1.0) < 1e-13
            assert (N >= -1e-15).all()
            k = O.find_span(U, p, u)
            off = np.ones(len(N), bool)
            off[k - p:k + 1] = False
            assert (N[off] == 0).all()


@pytest.mark.parametrize("p", range(1, 8))
def test_bernstein_closed_form(p):
    U = np.array([0.0] * (p + 1) + [1.0] * (p + 1))
    for u in np.linspace(0, 1, 17):
        N, _, dNdu = O.basis_dense(U, p, u)
        ref = [math.comb(p, i) * u ** i * (1 - u) ** (p - i) for i in range(p + 1)]
        dref = [math.comb(p, i) * (i * u ** (i - 1) * (1 - u) ** (p - i) if i else 0.0)
                - math.comb(p, i) * ((p - i) * u ** i * (1 - u) ** (p - i - 1) if i < p else 0.0)
                for i in range(p + 1)]
        np.testing.assert_allclose(N, ref, rtol=0, atol=1e-14)
        np.testing.assert_allclose(dNdu, dref, rtol=0, atol=1e-12)


def test_uniform_quadratic_and_cubic_pieces():
    # uniform integer knots; on the domain interval with local t in [0,1):
    # quadratic pieces (1-t)^2/2, (-2t^2+2t+1)/2, t^2/2
    # cubic pieces (1-t)^3/6, (3t^3-6t^2+4)/6, (-3t^3+3t^2+3t+1)/6, t^3/6
    U2 = np.arange(6, dtype=float)
    U3 = np.arange(8, dtype=float)
    for t in np.linspace(0, 0.95, 11):
        N2, _, _ = O.basis_dense(U2, 2, 2 + t)
        np.testing.assert_allclose(N2, [(1 - t) ** 2 / 2, (-2 * t * t + 2 * t + 1) / 2, t * t / 2],
                                   atol=1e-14)
        N3, _, _ = O.basis_dense(U3, 3, 3 + t)
        np.testing.assert_allclose(
            N3, [(1 - t) ** 3 / 6, (3 * t ** 3 - 6 * t * t + 4) / 6,
                 (-3 * t ** 3 + 3 * t * t + 3 * t + 1) / 6, t ** 3 / 6], atol=1e-14)


def test_continuity_at_simple_knots():
    g = rng(13)
    for _ in range(30):
        p = int(g.integers(1, 6))
        U = rand_knots(g, int(g.integers(p + 2, 14)), p)
        for kn in U[p + 1:len(U) - p - 1]:
            h = 1e-9
            a, _, da = O.basis_dense(U, p, kn - h)
            b, _, db = O.basis_dense(U, p, kn + h)
            # a jump would be O(1); a continuous function moves by at most
            # 2h times its steepest slope across the knot
            slope = max(np.abs(da).max(), np.abs(db).max())
            assert np.abs(a - b).max() <= 2.5 * h * slope + 1e-12


def test_basis_du_matches_finite_difference():
    g = rng(14)
    for _ in range(40):
        p = int(g.integers(1, 6))
        U = rand_knots(g, int(g.integers(p + 1, 14)), p)
        u = g.uniform(0.02, 0.98)
        if np.min(np.abs(U - u)) < 1e-4:
            continue
        h = 1e-6
        _, _, dd = O.basis_dense(U, p, u)
        fd = (O.basis_dense(U, p, u + h)[0] - O.basis_dense(U, p, u - h)[0]) / (2 * h)
        np.testing.assert_allclose(dd, fd, atol=1e-5 * max(1, np.abs(fd).max()))


def test_basis_knot_derivative_finite_difference_and_sum_rule():
    g = rng(15)
    for _ in range(40):
        p = int(g.integers(1, 6))
        U = rand_knots(g, int(g.integers(p + 2, 14)), p)
        u = g.uniform(0.02, 0.98)
        _, dU, du = O.basis_dense(U, p, u)
        # sum over all knots of dN/dU_k equals -dN/du (shift invariance)
        np.testing.assert_allclose(dU.sum(axis=1), -du, atol=1e-9 * max(1, np.abs(du).max()))
        # FD on interior simple knots away from u
        for k in range(p + 1, len(U) - p - 1):
            if np.min(np.abs(np.delete(U, k) - U[k])) < 1e-3 or abs(U[k] - u) < 1e-3:
                continue
            h = 1e-7
            Up, Um = U.copy(), U.copy()
            Up[k] += h
            Um[k] -= h
            fd = (O.basis_dense(Up, p, u)[0] - O.basis_dense(Um, p, u)[0]) / (2 * h)
            np.testing.assert_allclose(dU[:, k], fd, atol=2e-5 * max(1, np.abs(fd).max()))


def test_dense_equals_local_basis():
    g = rng(16)
    for _ in range(100):
        p = int(g.integers(1, 8))
        U = rand_knots(g, int(g.integers(p + 1, 16)), p, repeat=0.3)
        for u in np.concatenate([g.uniform(0, 1, 5), [0.0, 1.0], U[p:len(U) - p]]):
            N, dU, du = O.basis_dense(U, p, u)
            k, Nl, dUl, dul = O.basis_local(U, p, u)
            np.testing.assert_allclose(N[k - p:k + 1], Nl, atol=1e-15)
            np.testing.assert_allclose(du[k - p:k + 1], dul, atol=1e-12 * max(1, np.abs(du).max()))
            dense_win = dU[k - p:k + 1, k - p:k + p + 2]
            np.testing.assert_allclose(dense_win, dUl, atol=1e-12 * max(1, np.abs(dU).max()))
            # no knot outside the window influences the non-zero functions
            mask = np.ones(len(U), bool)
            mask[k - p:k + p + 2] = False
            assert np.abs(dU[k - p:k + 1][:, mask]).max(initial=0) == 0


# --------------------------------------------------------------------------
# forward: an independent evaluator (de Boor's algorithm on homogeneous points)
# --------------------------------------------------------------------------

def de_boor(U, p, Pw, u):
    """de Boor's corner cutting for one homogeneous curve (NURBS Book, A3.1
    style), with its own span from bisection."""
    n = len(U) - p - 2
    u = min(max(u, U[p]), U[n + 1])
    k = min(max(bisect.bisect_right(list(U), u) - 1, p), n)
    d = [np.array(Pw[j + k - p], float) for j in range(p + 1)]
    for r in range(1, p + 1):
        for j in range(p, r - 1, -1):
            lo = U[j + k - p]
            hi = U[j + 1 + k - r]
            a = (u - lo) / (hi - lo)
            d[j] = (1 - a) * d[j - 1] + a * d[j]
    return d[p]


def de_boor_surface(ctrl, w, ku, kv, p, q, us, vs):
    Pw = np.concatenate([ctrl * w[..., None], w[..., None]], axis=-1)
    out = np.zeros((len(us), len(vs), 3))
    for b, v in enumerate(vs):
        col = [de_boor(kv, q, Pw[i], v) for i in range(Pw.shape[0])]
        for a, u in enumerate(us):
            s = de_boor(ku, p, col, u)
            out[a, b] = s[:3] / s[3]
    return out


@pytest.mark.parametrize("seed", range(6))
def test_forward_matches_de_boor(seed):
    g = rng(100 + seed)
    p, q = int(g.integers(1, 6)), int(g.integers(1, 6))
    nu_c, nv_c = int(g.integers(p + 1, p + 8)), int(g.integers(q + 1, q + 8))
    ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c, repeat=0.25)
    us = np.concatenate([g.uniform(0, 1, 9), [0.0, 1.0], ku[p + 1:nu_c]])
    vs = np.concatenate([g.uniform(0, 1, 7), [0.0, 1.0], kv[q + 1:nv_c]])
    for local in (False, True):
        S = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, local=local)
        ref = de_boor_surface(ctrl, w, ku, kv, p, q, us, vs)
        np.testing.assert_allclose(S, ref, atol=1e-12)


def quarter_cylinder():
    ctrl = np.array([[[1, 0, 0], [1, 0, 1]], [[1, 1, 0], [1, 1, 1]], [[0, 1, 0], [0, 1, 1]]], float)
    w = np.array([[1, 1], [2 ** -0.5, 2 ** -0.5], [1, 1]])
    return ctrl, w, np.array([0, 0, 0, 1, 1, 1.]), np.array([0, 0, 1, 1.])


def test_quarter_circle_cylinder():
    ctrl, w, ku, kv = quarter_cylinder()
    us = np.linspace(0, 1, 33)
    vs = np.linspace(0, 1, 5)
    S = O.surface_fwd(ctrl, w, ku, kv, 2, 1, us, vs)
    np.testing.assert_allclose(S[..., 0] ** 2 + S[..., 1] ** 2, 1.0, atol=1e-14)
    np.testing.assert_allclose(S[..., 2], np.broadcast_to(vs, S.shape[:2]), atol=1e-15)
    mid = O.surface_fwd(ctrl, w, ku, kv, 2, 1, [0.5], [0.3])
    np.testing.assert_allclose(mid[0, 0, :2], [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    # the angle is monotone in u over the quarter
    ang = np.arctan2(S[:, 0, 1], S[:, 0, 0])
    assert (np.diff(ang) > 0).all() and abs(ang[0]) < 1e-15 and abs(ang[-1] - np.pi / 2) < 1e-14


def test_endpoint_interpolation():
    g = rng(17)
    for _ in range(10):
        p, q = int(g.integers(1, 6)), int(g.integers(1, 6))
        nu_c, nv_c = int(g.integers(p + 1, 12)), int(g.integers(q + 1, 12))
        ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c, repeat=0.3)
        S = O.surface_fwd(ctrl, w, ku, kv, p, q, [0.0, 1.0], [0.0, 1.0])
        np.testing.assert_allclose(S[0, 0], ctrl[0, 0], atol=1e-14)
        np.testing.assert_allclose(S[0, 1], ctrl[0, -1], atol=1e-14)
        np.testing.assert_allclose(S[1, 0], ctrl[-1, 0], atol=1e-14)
        np.testing.assert_allclose(S[1, 1], ctrl[-1, -1], atol=1e-14)


def test_weight_scale_and_equal_weights():
    g = rng(18)
    p, q, nu_c, nv_c = 3, 2, 9, 7
    ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c)
    us, vs = g.uniform(0, 1, 13), g.uniform(0, 1, 11)
    S1 = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs)
    S2 = O.surface_fwd(ctrl, 3.7 * w, ku, kv, p, q, us, vs)
    np.testing.assert_allclose(S1, S2, atol=1e-14)
    # equal weights: the non-rational B-spline, independent of the common weight
    Sa = O.surface_fwd(ctrl, np.full_like(w, 0.3), ku, kv, p, q, us, vs)
    Sb = O.surface_fwd(ctrl, np.ones_like(w), ku, kv, p, q, us, vs)
    np.testing.assert_allclose(Sa, Sb, atol=1e-14)
    ref = de_boor_surface(ctrl, np.ones_like(w), ku, kv, p, q, us, vs)
    np.testing.assert_allclose(Sb, ref, atol=1e-13)


def test_affine_invariance_and_convex_hull():
    g = rng(19)
    p, q, nu_c, nv_c = 2, 4, 8, 9
    ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c)
    us, vs = g.uniform(0, 1, 10), g.uniform(0, 1, 12)
    A = g.normal(size=(3, 3))
    t = g.normal(size=3)
    S = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs)
    S2 = O.surface_fwd(ctrl @ A.T + t, w, ku, kv, p, q, us, vs)
    np.testing.assert_allclose(S2, S @ A.T + t, atol=1e-13)
    # every point lies in the bounding box of its active (p+1)x(q+1) patch
    for a, u in enumerate(us):
        k = O.find_span(ku, p, u)
        for b, v in enumerate(vs):
            l = O.find_span(kv, q, v)
            patch = ctrl[k - p:k + 1, l - q:l + 1].reshape(-1, 3)
            assert (S[a, b] >= patch.min(0) - 1e-13).all()
            assert (S[a, b] <= patch.max(0) + 1e-13).all()


def test_parametric_derivative_matches_finite_difference():
    g = rng(20)
    p, q, nu_c, nv_c = 3, 2, 8, 6
    ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c)
    us, vs = g.uniform(0.05, 0.95, 6), g.uniform(0.05, 0.95, 5)
    _, Su, Sv = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, derivs=True)
    h = 1e-6
    fdu = (O.surface_fwd(ctrl, w, ku, kv, p, q, us + h, vs)
           - O.surface_fwd(ctrl, w, ku, kv, p, q, us - h, vs)) / (2 * h)
    fdv = (O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs + h)
           - O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs - h)) / (2 * h)
    np.testing.assert_allclose(Su, fdu, atol=1e-6)
    np.testing.assert_allclose(Sv, fdv, atol=1e-6)


def test_normals_of_cylinder_and_plane():
    """The quarter cylinder's unit normal is radial, (x, y, 0), pointing out
    (S_u runs along the arc counter-clockwise, S_v along +z); a net in the
    plane z = 0 with u along +x and v along +y has normal +z whatever its
    weights."""
    ctrl, w, ku, kv = quarter_cylinder()
    us, vs = np.linspace(0, 1, 17), np.linspace(0, 1, 4)
    S, Su, Sv = O.surface_fwd(ctrl, w, ku, kv, 2, 1, us, vs, derivs=True)
    n = O.normals(Su, Sv)
    np.testing.assert_allclose(n[..., :2], S[..., :2], atol=1e-13)
    np.testing.assert_allclose(n[..., 2], 0.0, atol=1e-15)
    g = rng(23)
    p, q, nu_c, nv_c = 3, 2, 7, 6
    i, j = np.meshgrid(np.arange(nu_c), np.arange(nv_c), indexing="ij")
    flat = np.stack([i / (nu_c - 1), j / (nv_c - 1), np.zeros(i.shape)], -1)
    flat[..., :2] += g.uniform(-0.05, 0.05, flat[..., :2].shape)
    w = g.uniform(0.5, 1.5, (nu_c, nv_c))
    _, Su, Sv = O.surface_fwd(flat, w, rand_knots(g, nu_c, p), rand_knots(g, nv_c, q), p, q,
                              g.uniform(0, 1, 9), g.uniform(0, 1, 8), derivs=True)
    np.testing.assert_allclose(O.normals(Su, Sv), np.broadcast_to([0, 0, 1.0], Su.shape), atol=1e-12)


# --------------------------------------------------------------------------
# gradients
# --------------------------------------------------------------------------

def loss_and_grad_setup(seed, p=3, q=2, nu_c=7, nv_c=6, nu_s=9, nv_s=8, repeat=0.0):
    g = rng(seed)
    ctrl, w, ku, kv = rand_surface(g, p, q, nu_c, nv_c, repeat)
    us, vs = np.sort(g.uniform(0, 1, nu_s)), np.sort(g.uniform(0, 1, nv_s))
    G = g.normal(size=(nu_s, nv_s, 3))
    return ctrl, w, ku, kv, p, q, us, vs, G


def lin_loss(ctrl, w, ku, kv, p, q, us, vs, G):
    return float((O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs) * G).sum())


@pytest.mark.parametrize("local", [False, True])
def test_grad_ctrl_and_weights_fd(local):
    ctrl, w, ku, kv, p, q, us, vs, G = loss_and_grad_setup(21)
    dP, dW, _, _ = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G, local=local)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 2), (6, 5), (2, 4)]:
        for x in range(3):
            cp, cm = ctrl.copy(), ctrl.copy()
            cp[i, j, x] += h
            cm[i, j, x] -= h
            fd = (lin_loss(cp, w, ku, kv, p, q, us, vs, G) - lin_loss(cm, w, ku, kv, p, q, us, vs, G)) / (2 * h)
            assert abs(dP[i, j, x] - fd) < 1e-7 * max(1, abs(fd))
        wp, wm = w.copy(), w.copy()
        wp[i, j] += h
        wm[i, j] -= h
        fd = (lin_loss(ctrl, wp, ku, kv, p, q, us, vs, G) - lin_loss(ctrl, wm, ku, kv, p, q, us, vs, G)) / (2 * h)
        assert abs(dW[i, j] - fd) < 1e-7 * max(1, abs(fd))


def test_grad_invariants_translation_and_weight_scale():
    ctrl, w, ku, kv, p, q, us, vs, G = loss_and_grad_setup(22, repeat=0.3)
    dP, dW, _, _ = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G)
    # S(P + t) = S(P) + t  =>  sum_ij dL/dP_ij = sum_pts dL/dS
    np.testing.assert_allclose(dP.sum(axis=(0, 1)), G.sum(axis=(0, 1)), atol=1e-12)
    # S(cW) = S(W)  =>  sum_ij w_ij dL/dw_ij = 0
    assert abs((w * dW).sum()) < 1e-12 * np.abs(w * dW).sum()


@pytest.mark.parametrize("local", [False, True])
def test_grad_knots_fd(local):
    ctrl, w, ku, kv, p, q, us, vs, G = loss_and_grad_setup(23, nu_c=9, nv_c=8, nu_s=12, nv_s=11)
    _, _, dU, dV = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G, local=local)
    h = 1e-7
    checked = 0
    for knots, deg, dK, which in ((ku, p, dU, 0), (kv, q, dV, 1)):
        samples = us if which == 0 else vs
        for k in range(deg + 1, len(knots) - deg - 1):
            if np.min(np.abs(samples - knots[k])) < 1e-4:
                continue
            kp, km = knots.copy(), knots.copy()
            kp[k] += h
            km[k] -= h
            if which == 0:
                fd = (lin_loss(ctrl, w, kp, kv, p, q, us, vs, G) - lin_loss(ctrl, w, km, kv, p, q, us, vs, G)) / (2 * h)
            else:
                fd = (lin_loss(ctrl, w, ku, kp, p, q, us, vs, G) - lin_loss(ctrl, w, ku, km, p, q, us, vs, G)) / (2 * h)
            assert abs(dK[k] - fd) < 1e-5 * max(1, abs(fd)), (which, k, dK[k], fd)
            checked += 1
    assert checked >= 6


def test_grad_knots_shift_and_scale_invariance():
    ctrl, w, ku, kv, p, q, us, vs, G = loss_and_grad_setup(24, nu_c=9, nv_c=8, repeat=0.3)
    _, _, dU, dV = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G)
    _, Su, Sv = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, derivs=True)
    gSu = (G * Su).sum(axis=2)
    gSv = (G * Sv).sum(axis=2)
    # N(u + c; U + c) = N(u; U):  sum_k dL/dU_k = -sum g . S_u
    np.testing.assert_allclose(dU.sum(), -gSu.sum(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(dV.sum(), -gSv.sum(), rtol=1e-10, atol=1e-10)
    # N(l u; l U) = N(u; U):  sum_k U_k dL/dU_k = -sum g . u S_u
    np.testing.assert_allclose((ku * dU).sum(), -(gSu * us[:, None]).sum(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose((kv * dV).sum(), -(gSv * vs[None, :]).sum(), rtol=1e-10, atol=1e-10)


def test_grad_knots_bezier_closed_form():
    # knots [a^{p+1}, b^{p+1}]: S(u) = Bezier((u-a)/(b-a)), so moving all
    # copies of a gives sum_copies dL/dU = sum g . S_t (u-b)/(b-a)^2
    g = rng(25)
    p, q = 3, 2
    a, b = 0.0, 1.0
    ctrl = g.uniform(-1, 1, (p + 1, q + 1, 3))
    w = g.uniform(0.5, 1.5, (p + 1, q + 1))
    ku = np.array([a] * (p + 1) + [b] * (p + 1))
    kv = np.array([0.0] * (q + 1) + [1.0] * (q + 1))
    us, vs = np.linspace(0, 1, 7), np.linspace(0, 1, 5)
    G = g.normal(size=(7, 5, 3))
    _, _, dU, _ = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G)
    _, Su, _ = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, derivs=True)
    St = Su * (b - a)
    expect_a = ((G * St).sum(axis=2) * ((us - b) / (b - a) ** 2)[:, None]).sum()
    expect_b = ((G * St).sum(axis=2) * (-(us - a) / (b - a) ** 2)[:, None]).sum()
    np.testing.assert_allclose(dU[:p + 1].sum(), expect_a, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(dU[p + 1:].sum(), expect_b, rtol=1e-11, atol=1e-12)


def test_dense_equals_local_surface():
    for seed in range(4):
        ctrl, w, ku, kv, p, q, us, vs, G = loss_and_grad_setup(30 + seed, p=1 + seed, q=4 - seed % 3,
                                                                nu_c=8, nv_c=7, repeat=0.3)
        S0 = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs)
        S1 = O.surface_fwd(ctrl, w, ku, kv, p, q, us, vs, local=True)
        np.testing.assert_allclose(S0, S1, atol=1e-14)
        r0 = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G)
        r1 = O.surface_bwd(ctrl, w, ku, kv, p, q, us, vs, G, local=True)
        for x0, x1 in zip(r0, r1):
            np.testing.assert_allclose(x0, x1, rtol=0, atol=1e-13 * max(1, np.abs(x0).max()))
