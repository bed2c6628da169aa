"""Pins for the oracle's curve functions (eq. NURBS with one parametric
direction dropped, Sec. 3; derivatives as Sec. 3.2.1 without v).

* the exact rational quarter circle (weights 1, sqrt(2)/2, 1);
* the rational Bezier closed form from Bernstein polynomials built with
  binomial coefficients (no recursion);
* a curve equals the v = 0 edge of a degree-1-in-v surface whose two control
  columns both carry the curve (points, and every gradient) -- the surface
  oracle is separate code;
* central finite differences for dC/du, dL/dP, dL/dw and interior knots;
* translation invariance (sum dP = sum g), projective invariance
  (sum w dW = 0), knot shift and scale invariance
  (sum dU = -sum g.C_u, sum U dU = -sum g.u C_u).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rand_curve(g, p, nc, dim, repeat=0.0):
    inner = np.sort(g.uniform(0.05, 0.95, nc - p - 1))
    if repeat > 0 and len(inner) > 1:
        m = 1
        for t in range(1, len(inner)):
            if g.uniform() < repeat and m < p:
                inner[t] = inner[t - 1]
                m += 1
            else:
                m = 1
    U = np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])
    return g.uniform(-1, 1, (nc, dim)), g.uniform(0.5, 1.5, nc), U


def test_quarter_circle():
    c = np.array([[1, 0], [1, 1], [0, 1.]])
    w = np.array([1, 2 ** -0.5, 1])
    us = np.linspace(0, 1, 41)
    C = O.curve_eval(c, w, [0, 0, 0, 1, 1, 1], 2, us)
    np.testing.assert_allclose(np.hypot(C[:, 0], C[:, 1]), 1.0, atol=1e-15)
    np.testing.assert_allclose(O.curve_eval(c, w, [0, 0, 0, 1, 1, 1], 2, [0.5])[0], [2 ** -0.5] * 2, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_rational_bezier_closed_form(p):
    g = rng(40 + p)
    c, w, _ = rand_curve(g, p, p + 1, 3)
    U = np.concatenate([np.zeros(p + 1), np.ones(p + 1)])
    us = np.concatenate([g.uniform(0, 1, 20), [0.0, 1.0]])
    B = np.array([[math.comb(p, i) * u ** i * (1 - u) ** (p - i) for i in range(p + 1)] for u in us])
    ref = (B * w) @ c / (B @ w)[:, None]
    np.testing.assert_allclose(O.curve_eval(c, w, U, p, us), ref, atol=1e-13)


def as_surface(c, w):
    """The degree-1-in-v surface whose two columns carry the curve (z lifted
    by 1 on the second column)."""
    nc = len(c)
    c3 = np.zeros((nc, 3))
    c3[:, :c.shape[1]] = c
    ctrl = np.stack([c3, c3 + [0, 0, 1.0]], axis=1)
    return ctrl, np.stack([w, w], axis=1), np.array([0, 0, 1, 1.0])


@pytest.mark.parametrize("seed", range(4))
def test_curve_is_surface_edge(seed):
    g = rng(50 + seed)
    p = int(g.integers(1, 6))
    nc = int(g.integers(p + 1, p + 9))
    c, w, U = rand_curve(g, p, nc, 3, repeat=0.3)
    us = np.sort(np.concatenate([g.uniform(0, 1, 15), U[p + 1:nc], [0.0, 1.0]]))
    C = O.curve_eval(c, w, U, p, us)
    ctrl, ws, kv = as_surface(c, w)
    S = O.surface_fwd(ctrl, ws, U, kv, p, 1, us, [0.0])
    np.testing.assert_allclose(S[:, 0, :], C, atol=1e-13)
    G = g.normal(size=(len(us), 3))
    dP, dW, dU = O.curve_grad(c, w, U, p, us, G)
    sP, sW, sU, _ = O.surface_bwd(ctrl, ws, U, kv, p, 1, us, [0.0], G[:, None, :])
    np.testing.assert_allclose(dP, sP[:, 0], atol=1e-12)
    np.testing.assert_allclose(dW, sW[:, 0], atol=1e-12)
    np.testing.assert_allclose(dU, sU, atol=1e-11)


def test_finite_differences():
    g = rng(60)
    p, nc, dim = 3, 9, 2
    c, w, U = rand_curve(g, p, nc, dim)
    us = np.sort(g.uniform(0.02, 0.98, 30))
    G = g.normal(size=(len(us), dim))
    L = lambda c_, w_, U_: float((O.curve_eval(c_, w_, U_, p, us) * G).sum())
    dP, dW, dU = O.curve_grad(c, w, U, p, us, G)
    h = 1e-6
    for i in range(nc):
        for x in range(dim):
            e = np.zeros_like(c)
            e[i, x] = h
            assert abs((L(c + e, w, U) - L(c - e, w, U)) / (2 * h) - dP[i, x]) < 1e-7
        e = np.zeros_like(w)
        e[i] = h
        assert abs((L(c, w + e, U) - L(c, w - e, U)) / (2 * h) - dW[i]) < 1e-6
    for k in range(p + 1, nc):  # interior knots, simple, no sample nearby
        if np.min(np.abs(us - U[k])) < 1e-4:
            continue
        e = np.zeros_like(U)
        e[k] = 1e-7
        fd = (L(c, w, U + e) - L(c, w, U - e)) / 2e-7
        assert abs(fd - dU[k]) < 1e-5 * max(1.0, abs(dU[k])), (k, fd, dU[k])
    C, Cu = O.curve_eval(c, w, U, p, us, derivs=True)
    fdu = (O.curve_eval(c, w, U, p, us + 1e-6) - O.curve_eval(c, w, U, p, us - 1e-6)) / 2e-6
    np.testing.assert_allclose(Cu, fdu, atol=1e-6)


def test_invariants():
    g = rng(61)
    p, nc, dim = 4, 11, 3
    c, w, U = rand_curve(g, p, nc, dim, repeat=0.3)
    us = np.sort(g.uniform(0, 1, 50))
    G = g.normal(size=(len(us), dim))
    dP, dW, dU = O.curve_grad(c, w, U, p, us, G)
    np.testing.assert_allclose(dP.sum(0), G.sum(0), atol=1e-12)
    assert abs((w * dW).sum()) < 1e-12
    _, Cu = O.curve_eval(c, w, U, p, us, derivs=True)
    np.testing.assert_allclose(dU.sum(), -(G * Cu).sum(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose((U * dU).sum(), -(G * Cu * us[:, None]).sum(), rtol=1e-10, atol=1e-10)
