"""ctypes wrapper around the FP64 CPU oracle (``nurbs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package's smoke
check and by the benchmark's CPU-baseline leg, never by the product path.
It shares no code with the HIP implementation; inputs come from the seeded
generators as float32 and are widened here to float64.

Paper passages followed (NURBS-Diff, arXiv 2104.14547): eq. (NURBS) and
eq. (NURBSBasis) with the indicator eq. (BSplineBasis2) for the forward map
(Sec. 3.1); eqs. (NURBSuDerivative4), (NURBSvDerivative5),
(NURBSvDerivative6) and the knot-derivative recursion of Sec. 3.2.1 for the
backward; eq. (NURBSuDerivative1) of Appendix A for dS/du.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nurbs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_fp = ctypes.POINTER(ctypes.c_float)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math), OpenMP on."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        L.oracle_find_span.restype = ctypes.c_int
        L.oracle_find_span.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.oracle_basis_dense.restype = ctypes.c_int
        L.oracle_basis_dense.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         _dp, _dp, _dp]
        L.oracle_basis_local.restype = ctypes.c_int
        L.oracle_basis_local.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         _dp, _dp, _dp]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_fwd.restype = ctypes.c_int
        L.oracle_fwd.argtypes = [ctypes.c_int, _ip, _lp] + [_dp] * 9 + [ctypes.c_int, ctypes.c_int]
        L.oracle_bwd.restype = ctypes.c_int
        L.oracle_bwd.argtypes = [ctypes.c_int, _ip, _lp] + [_dp] * 11 + [ctypes.c_int, ctypes.c_int]
        L.oracle_curve_fwd.restype = ctypes.c_int
        L.oracle_curve_fwd.argtypes = [ctypes.c_int, _ip, _lp] + [_dp] * 6 + [ctypes.c_int]
        L.oracle_curve_bwd.restype = ctypes.c_int
        L.oracle_curve_bwd.argtypes = [ctypes.c_int, _ip, _lp] + [_dp] * 8 + [ctypes.c_int]
        L.oracle_scattered_fwd.restype = ctypes.c_int
        L.oracle_scattered_fwd.argtypes = [ctypes.c_int] * 5 + [_dp] * 8 + [ctypes.c_int]
        L.oracle_scattered_bwd.restype = ctypes.c_int
        L.oracle_scattered_bwd.argtypes = [ctypes.c_int] * 5 + [_dp] * 10 + [ctypes.c_int]
        L.oracle_nearest.restype = ctypes.c_int
        L.oracle_nearest.argtypes = [ctypes.c_int, _fp, ctypes.c_int, _fp, ctypes.c_int, _ip, _fp, ctypes.c_int]
        L.oracle_chamfer_hausdorff.restype = ctypes.c_int
        L.oracle_chamfer_hausdorff.argtypes = [ctypes.c_int, _fp, ctypes.c_int, _fp, ctypes.c_int, _dp, _dp, _dp,
                                               ctypes.c_int]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _d(x):
    """float64 contiguous copy + pointer (keeps the array alive via return)."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _null():
    return ctypes.cast(None, _dp)


def find_span(U, p: int, u: float) -> int:
    Ua, Up = _d(U)
    return int(lib().oracle_find_span(Up, len(Ua), int(p), float(u)))


def basis_dense(U, p: int, u: float):
    """(N[n+1], dN/dU[n+1][len U], dN/du[n+1]) of every degree-p function."""
    Ua, Up = _d(U)
    nc = len(Ua) - p - 1
    N = np.zeros(nc)
    dU = np.zeros((nc, len(Ua)))
    du = np.zeros(nc)
    rc = lib().oracle_basis_dense(Up, len(Ua), int(p), float(u), N.ctypes.data_as(_dp),
                                  dU.ctypes.data_as(_dp), du.ctypes.data_as(_dp))
    if rc:
        raise OracleError(rc)
    return N, dU, du


def basis_local(U, p: int, u: float):
    """(span k, N[p+1], dN/dU[p+1][2p+2] over knots k-p..k+p+1, dN/du[p+1])."""
    Ua, Up = _d(U)
    N = np.zeros(p + 1)
    dU = np.zeros((p + 1, 2 * p + 2))
    du = np.zeros(p + 1)
    k = lib().oracle_basis_local(Up, len(Ua), int(p), float(u), N.ctypes.data_as(_dp),
                                 dU.ctypes.data_as(_dp), du.ctypes.data_as(_dp))
    return int(k), N, dU, du


def _batch_args(b):
    shapes = np.ascontiguousarray(b.shapes, np.int32)
    offs = np.ascontiguousarray(b.offsets, np.int64)
    keep = [shapes, offs]
    ptrs = []
    for name in ("ctrl", "w", "ku", "kv", "us", "vs"):
        a, p = _d(getattr(b, name))
        keep.append(a)
        ptrs.append(p)
    return keep, shapes.ctypes.data_as(_ip), offs.ctypes.data_as(_lp), ptrs


def n_pts_floats(b) -> int:
    s = np.asarray(b.shapes, np.int64)
    o = np.asarray(b.offsets, np.int64)
    if len(s) == 0:
        return 0
    return int((o[:, 6] + s[:, 4] * s[:, 5] * 3).max())


def fwd(b, local: bool = False, nthreads: int = 0, derivs: bool = False):
    """Surface points (float64, packed pts layout) of a packed batch ``b``.

    With ``derivs`` also returns dS/du and dS/dv at every sample."""
    keep, sh, of, ptrs = _batch_args(b)
    npf = n_pts_floats(b)
    pts = np.zeros(npf)
    du = np.zeros(npf) if derivs else None
    dv = np.zeros(npf) if derivs else None
    rc = lib().oracle_fwd(len(b.shapes), sh, of, *ptrs, pts.ctypes.data_as(_dp),
                          du.ctypes.data_as(_dp) if derivs else _null(),
                          dv.ctypes.data_as(_dp) if derivs else _null(),
                          int(bool(local)), int(nthreads))
    del keep
    if rc:
        raise OracleError(rc)
    return (pts, du, dv) if derivs else pts


def bwd(b, grad_pts, local: bool = False, nthreads: int = 0):
    """(dL/dctrl, dL/dw, dL/dku, dL/dkv) in the packed layout, float64."""
    keep, sh, of, ptrs = _batch_args(b)
    g, gp = _d(grad_pts)
    gc = np.zeros(len(b.ctrl))
    gw = np.zeros(len(b.w))
    gku = np.zeros(len(b.ku))
    gkv = np.zeros(len(b.kv))
    rc = lib().oracle_bwd(len(b.shapes), sh, of, *ptrs, gp, gc.ctypes.data_as(_dp),
                          gw.ctypes.data_as(_dp), gku.ctypes.data_as(_dp),
                          gkv.ctypes.data_as(_dp), int(bool(local)), int(nthreads))
    del keep, g
    if rc:
        raise OracleError(rc)
    return gc, gw, gku, gkv


class _One:
    """A one-surface packed batch built from dense arrays (oracle-side helper)."""

    def __init__(self, ctrl, w, ku, kv, p, q, us, vs):
        ctrl = np.asarray(ctrl, np.float64)
        nu_c, nv_c = ctrl.shape[:2]
        us = np.atleast_1d(np.asarray(us, np.float64))
        vs = np.atleast_1d(np.asarray(vs, np.float64))
        self.shapes = np.array([[p, q, nu_c, nv_c, len(us), len(vs)]], np.int32)
        self.offsets = np.zeros((1, 7), np.int64)
        self.ctrl = ctrl.ravel()
        self.w = np.asarray(w, np.float64).ravel()
        self.ku = np.asarray(ku, np.float64)
        self.kv = np.asarray(kv, np.float64)
        self.us, self.vs = us, vs
        self.dims = (nu_c, nv_c, len(us), len(vs))


def surface_fwd(ctrl, w, ku, kv, p, q, us, vs, local=False, derivs=False):
    """Dense-array convenience: returns S[nu_s][nv_s][3] (and S_u, S_v)."""
    one = _One(ctrl, w, ku, kv, p, q, us, vs)
    nu_c, nv_c, nu_s, nv_s = one.dims
    r = fwd(one, local=local, derivs=derivs)
    if derivs:
        return tuple(x.reshape(nu_s, nv_s, 3) for x in r)
    return r.reshape(nu_s, nv_s, 3)


def surface_bwd(ctrl, w, ku, kv, p, q, us, vs, grad_pts, local=False):
    """Dense-array convenience: returns (dP[nu_c][nv_c][3], dW, dU, dV)."""
    one = _One(ctrl, w, ku, kv, p, q, us, vs)
    nu_c, nv_c, nu_s, nv_s = one.dims
    gc, gw, gku, gkv = bwd(one, np.asarray(grad_pts, np.float64).ravel(), local=local)
    return gc.reshape(nu_c, nv_c, 3), gw.reshape(nu_c, nv_c), gku, gkv


# --------------------------------------------------------------------------
# curves: eq. (NURBS) with one parametric direction dropped (Sec. 3)
# --------------------------------------------------------------------------

def _curve_args(cb):
    shapes = np.ascontiguousarray(cb.shapes, np.int32)
    offs = np.ascontiguousarray(cb.offsets, np.int64)
    keep = [shapes, offs]
    ptrs = []
    for name in ("ctrl", "w", "knots", "us"):
        a, p = _d(getattr(cb, name))
        keep.append(a)
        ptrs.append(p)
    return keep, shapes.ctypes.data_as(_ip), offs.ctypes.data_as(_lp), ptrs


def _curve_pts_len(cb):
    s = np.asarray(cb.shapes, np.int64)
    o = np.asarray(cb.offsets, np.int64)
    return int((o[:, 4] + s[:, 2] * s[:, 3]).max()) if len(s) else 0


def curve_fwd(cb, derivs: bool = False, nthreads: int = 0):
    """Curve points (packed [ns][dim] per curve, float64) of a packed curve
    batch ``cb`` (shapes (p, nc, ns, dim), offsets (ctrl, w, knots, us, pts));
    with ``derivs`` also dC/du."""
    keep, sh, of, ptrs = _curve_args(cb)
    n = _curve_pts_len(cb)
    pts = np.zeros(n)
    du = np.zeros(n) if derivs else None
    rc = lib().oracle_curve_fwd(len(cb.shapes), sh, of, *ptrs, pts.ctypes.data_as(_dp),
                                du.ctypes.data_as(_dp) if derivs else _null(), int(nthreads))
    del keep
    if rc:
        raise OracleError(rc)
    return (pts, du) if derivs else pts


def curve_bwd(cb, grad_pts, nthreads: int = 0):
    """(dL/dctrl, dL/dw, dL/dknots) of a packed curve batch, float64."""
    keep, sh, of, ptrs = _curve_args(cb)
    g, gp = _d(grad_pts)
    gc, gw, gk = np.zeros(len(cb.ctrl)), np.zeros(len(cb.w)), np.zeros(len(cb.knots))
    rc = lib().oracle_curve_bwd(len(cb.shapes), sh, of, *ptrs, gp, gc.ctypes.data_as(_dp),
                                gw.ctypes.data_as(_dp), gk.ctypes.data_as(_dp), int(nthreads))
    del keep, g
    if rc:
        raise OracleError(rc)
    return gc, gw, gk


class _OneCurve:
    def __init__(self, ctrl, w, U, p, us):
        ctrl = np.asarray(ctrl, np.float64)
        nc, dim = ctrl.shape
        us = np.atleast_1d(np.asarray(us, np.float64))
        self.shapes = np.array([[p, nc, len(us), dim]], np.int32)
        self.offsets = np.zeros((1, 5), np.int64)
        self.ctrl, self.w = ctrl.ravel(), np.asarray(w, np.float64).ravel()
        self.knots, self.us = np.asarray(U, np.float64), us
        self.dims = (nc, len(us), dim)


def curve_eval(ctrl, w, U, p, us, derivs=False):
    """Dense-array convenience: C[ns][dim] (and dC/du) of one curve."""
    one = _OneCurve(ctrl, w, U, p, us)
    nc, ns, dim = one.dims
    r = curve_fwd(one, derivs=derivs)
    if derivs:
        return r[0].reshape(ns, dim), r[1].reshape(ns, dim)
    return r.reshape(ns, dim)


def curve_grad(ctrl, w, U, p, us, G):
    """Dense-array convenience: (dP[nc][dim], dW[nc], dU[nc+p+1]) of one curve."""
    one = _OneCurve(ctrl, w, U, p, us)
    nc, ns, dim = one.dims
    gc, gw, gk = curve_bwd(one, np.asarray(G, np.float64).ravel())
    return gc.reshape(nc, dim), gw, gk


def normals(Su, Sv):
    """Unit normals (S_u x S_v) / |S_u x S_v| from the oracle's parametric
    derivatives (Appendix A, eq. NURBSuDerivative1); offset surfaces move
    points along them (Sec. 4.3).  (0, 0, 0) where the cross product is 0."""
    c = np.cross(np.asarray(Su, np.float64), np.asarray(Sv, np.float64))
    n = np.linalg.norm(c, axis=-1, keepdims=True)
    return np.where(n > 0, c / np.where(n > 0, n, 1.0), 0.0)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# --------------------------------------------------------------------------
# point-set losses: Sec. 4, eqs. (ChamferDistance), (HausdorffDistance)
# --------------------------------------------------------------------------

def _f32(x, dim):
    a = np.ascontiguousarray(np.asarray(x, np.float32).reshape(-1, dim))
    return a, a.ctypes.data_as(_fp)


def nearest(P, Q, nthreads: int = 0):
    """For each row of P [n][dim] the index of its nearest row of Q [m][dim]
    and that squared distance, decided in float32 (first index wins ties)."""
    dim = np.asarray(P).shape[-1]
    P, pp = _f32(P, dim)
    Q, qp = _f32(Q, dim)
    idx = np.zeros(len(P), np.int32)
    d2 = np.zeros(len(P), np.float32)
    rc = lib().oracle_nearest(dim, pp, len(P), qp, len(Q), idx.ctypes.data_as(_ip), d2.ctypes.data_as(_fp),
                              int(nthreads))
    if rc:
        raise OracleError(rc)
    return idx, d2


def chamfer_hausdorff(P, Q, nthreads: int = 0):
    """(CD, HD, dCD/dP [n][dim], dHD/dP [n][dim]) in float64."""
    dim = np.asarray(P).shape[-1]
    P, pp = _f32(P, dim)
    Q, qp = _f32(Q, dim)
    out = np.zeros(2)
    gcd = np.zeros((len(P), dim))
    ghd = np.zeros((len(P), dim))
    rc = lib().oracle_chamfer_hausdorff(dim, pp, len(P), qp, len(Q), out.ctypes.data_as(_dp),
                                        gcd.ctypes.data_as(_dp), ghd.ctypes.data_as(_dp), int(nthreads))
    if rc:
        raise OracleError(rc)
    return float(out[0]), float(out[1]), gcd, ghd


# --------------------------------------------------------------------------
# surfaces at scattered (u, v) pairs: eq. (NURBS) at each pair
# --------------------------------------------------------------------------

def scattered_fwd(ctrl, w, ku, kv, p, q, uv, derivs=False, local=True):
    """S [npts][3] (and S_u, S_v) of one surface at the pairs uv [npts][2]."""
    ctrl = np.asarray(ctrl, np.float64)
    nu_c, nv_c = ctrl.shape[:2]
    uv = np.ascontiguousarray(np.asarray(uv, np.float64).reshape(-1, 2))
    n = len(uv)
    S = np.zeros((n, 3))
    Su = np.zeros((n, 3)) if derivs else None
    Sv = np.zeros((n, 3)) if derivs else None
    keep = [_d(ctrl.ravel()), _d(np.asarray(w, np.float64).ravel()), _d(ku), _d(kv), _d(uv.ravel())]
    rc = lib().oracle_scattered_fwd(int(p), int(q), nu_c, nv_c, n, *[k[1] for k in keep],
                                    S.ctypes.data_as(_dp), Su.ctypes.data_as(_dp) if derivs else _null(),
                                    Sv.ctypes.data_as(_dp) if derivs else _null(), int(bool(local)))
    del keep
    if rc:
        raise OracleError(rc)
    return (S, Su, Sv) if derivs else S


def scattered_bwd(ctrl, w, ku, kv, p, q, uv, G, local=True):
    """(dP [nu_c][nv_c][3], dW [nu_c][nv_c], dU, dV) of one surface at the pairs uv."""
    ctrl = np.asarray(ctrl, np.float64)
    nu_c, nv_c = ctrl.shape[:2]
    uv = np.ascontiguousarray(np.asarray(uv, np.float64).reshape(-1, 2))
    n = len(uv)
    dP, dW = np.zeros((nu_c, nv_c, 3)), np.zeros((nu_c, nv_c))
    dU, dV = np.zeros(nu_c + p + 1), np.zeros(nv_c + q + 1)
    keep = [_d(ctrl.ravel()), _d(np.asarray(w, np.float64).ravel()), _d(ku), _d(kv), _d(uv.ravel()),
            _d(np.asarray(G, np.float64).ravel())]
    rc = lib().oracle_scattered_bwd(int(p), int(q), nu_c, nv_c, n, *[k[1] for k in keep],
                                    *[a.ctypes.data_as(_dp) for a in (dP, dW, dU, dV)], int(bool(local)))
    del keep
    if rc:
        raise OracleError(rc)
    return dP, dW, dU, dV
