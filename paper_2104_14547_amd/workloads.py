"""Seeded synthetic workloads for batched NURBS surface evaluation.

This module only *draws inputs*: control nets, weights, knot vectors,
parameter grids, targets and upstream gradients.  It holds none of the
method's arithmetic (no span search, no basis, no surface sum), so both the
HIP path and the FP64 oracle can consume it without sharing code.

Every random value is drawn in float64 from numpy's PCG64 generator and then
rounded once to float32.  The oracle widens the *same* float32 values to
float64, so both sides see bit-identical inputs.

Packed ("ragged") layout, used for every batch:
  ``shapes[s]  = (p, q, nu_c, nv_c, nu_s, nv_s)``            int32
  ``offsets[s] = (ctrl, w, ku, kv, us, vs, pts)`` element offsets, int64
  ``ctrl``  float32, surface s at ``ctrl[off:off + nu_c*nv_c*3]``, row-major
            ``[nu_c][nv_c][xyz]``
  ``w``     float32 ``[nu_c][nv_c]``
  ``ku/kv`` float32 knot vectors of length ``nu_c+p+1`` / ``nv_c+q+1``
  ``us/vs`` float32 parameter samples of length ``nu_s`` / ``nv_s``
  ``pts``   float32 ``[nu_s][nv_s][xyz]`` (outputs, targets, upstream grads)

Workload recipes (the paper's datasets are absent; these stand in for the
analytic-surface fitting experiments of the paper's surface-fitting section
and for its timing tables' control-net / sample-grid / degree sweeps):

* ``single_bicubic`` -- one 8x8 bicubic surface on a lattice, 64x64 samples.
* ``batch_bicubic``  -- 256 bicubic 16x16 surfaces, non-uniform clamped knots,
  128x128 samples each.
* ``fit_target``     -- the 64x64-control, 512x512-sample fitting problem
  towards z = sin(3x) cos(3y).
* ``uneven_batch``   -- 4096 surfaces, degrees 1..5, control sides 4..48 and
  sample sides 16..256 log-uniform, 10% repeated interior knots.
* ``curve_batch``    -- B curves in the plane or in space on jittered circles.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SHAPE_FIELDS = ("p", "q", "nu_c", "nv_c", "nu_s", "nv_s")
OFFSET_FIELDS = ("ctrl", "w", "ku", "kv", "us", "vs", "pts")


@dataclasses.dataclass
class Batch:
    """A packed batch of NURBS surfaces (float32 inputs, see module doc)."""

    name: str
    shapes: np.ndarray  # int32 [n][6]
    offsets: np.ndarray  # int64 [n][7]
    ctrl: np.ndarray
    w: np.ndarray
    ku: np.ndarray
    kv: np.ndarray
    us: np.ndarray
    vs: np.ndarray
    n_pts_floats: int
    target: np.ndarray | None = None  # float32, pts layout
    upstream: np.ndarray | None = None  # float32, pts layout (dL/dS)

    @property
    def n(self) -> int:
        return int(self.shapes.shape[0])

    @property
    def n_points(self) -> int:
        s = self.shapes.astype(np.int64)
        return int((s[:, 4] * s[:, 5]).sum())

    def surface(self, s: int) -> dict:
        """Views of surface ``s`` reshaped to their natural dense shapes."""
        p, q, nu_c, nv_c, nu_s, nv_s = (int(x) for x in self.shapes[s])
        o = [int(x) for x in self.offsets[s]]
        d = dict(
            p=p, q=q, nu_c=nu_c, nv_c=nv_c, nu_s=nu_s, nv_s=nv_s,
            ctrl=self.ctrl[o[0]:o[0] + nu_c * nv_c * 3].reshape(nu_c, nv_c, 3),
            w=self.w[o[1]:o[1] + nu_c * nv_c].reshape(nu_c, nv_c),
            ku=self.ku[o[2]:o[2] + nu_c + p + 1],
            kv=self.kv[o[3]:o[3] + nv_c + q + 1],
            us=self.us[o[4]:o[4] + nu_s],
            vs=self.vs[o[5]:o[5] + nv_s],
        )
        for key in ("target", "upstream"):
            arr = getattr(self, key)
            if arr is not None:
                d[key] = arr[o[6]:o[6] + nu_s * nv_s * 3].reshape(nu_s, nv_s, 3)
        return d

    def subset(self, idx) -> "Batch":
        """A new packed batch holding surfaces ``idx`` (in that order)."""
        parts = [self.surface(int(s)) for s in idx]
        return pack(self.name + "[subset]", parts)


def pack(name: str, parts: list[dict]) -> Batch:
    """Pack a list of per-surface dicts (keys as ``Batch.surface``)."""
    n = len(parts)
    shapes = np.zeros((n, 6), np.int32)
    offsets = np.zeros((n, 7), np.int64)
    cur = np.zeros(7, np.int64)
    bufs = {k: [] for k in ("ctrl", "w", "ku", "kv", "us", "vs")}
    tgt, ups = [], []
    for s, d in enumerate(parts):
        shapes[s] = [d[k] for k in SHAPE_FIELDS]
        offsets[s] = cur
        for k in bufs:
            bufs[k].append(np.ascontiguousarray(d[k], np.float32).ravel())
        sizes = [d["nu_c"] * d["nv_c"] * 3, d["nu_c"] * d["nv_c"],
                 d["nu_c"] + d["p"] + 1, d["nv_c"] + d["q"] + 1,
                 d["nu_s"], d["nv_s"], d["nu_s"] * d["nv_s"] * 3]
        cur = cur + np.asarray(sizes, np.int64)
        if "target" in d:
            tgt.append(np.ascontiguousarray(d["target"], np.float32).ravel())
        if "upstream" in d:
            ups.append(np.ascontiguousarray(d["upstream"], np.float32).ravel())
    cat = {k: (np.concatenate(v) if v else np.zeros(0, np.float32))
           for k, v in bufs.items()}
    return Batch(
        name=name, shapes=shapes, offsets=offsets, n_pts_floats=int(cur[6]),
        target=np.concatenate(tgt) if len(tgt) == n and n else None,
        upstream=np.concatenate(ups) if len(ups) == n and n else None,
        **cat)


def uniform_grid(n: int) -> np.ndarray:
    """Samples a/(n-1), a = 0..n-1, computed in float64, rounded once."""
    if n == 1:
        return np.zeros(1, np.float32)
    return (np.arange(n, dtype=np.float64) / (n - 1)).astype(np.float32)


def clamped_uniform_knots(n_ctrl: int, p: int) -> np.ndarray:
    """[0]*(p+1), k/(n_ctrl-p) for k=1..n_ctrl-p-1, [1]*(p+1)."""
    n_int = n_ctrl - p - 1
    inner = np.arange(1, n_int + 1, dtype=np.float64) / (n_int + 1)
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]).astype(np.float32)


def _interior_knots(rng: np.random.Generator, n_int: int, p: int,
                    repeat_prob: float) -> np.ndarray:
    """Sorted U(0,1) interior knots, rounded to float32 strictly inside (0,1).

    With ``repeat_prob`` > 0 each interior knot after the first is, with that
    probability, made equal to its predecessor, provided the multiplicity
    stays at most ``p``.
    """
    vals = np.sort(rng.uniform(0.0, 1.0, n_int))
    f = vals.astype(np.float32)
    for t in range(n_int):
        while f[t] <= 0.0 or f[t] >= 1.0:  # redraw a value that rounds onto the ends
            f[t] = np.float32(rng.uniform(0.0, 1.0))
    f = np.sort(f)
    if repeat_prob > 0.0 and n_int > 1:
        flips = rng.uniform(0.0, 1.0, n_int) < repeat_prob
        mult = 1
        for t in range(1, n_int):
            if flips[t] and mult < p:
                f[t] = f[t - 1]
                mult += 1
            elif f[t] == f[t - 1]:
                mult += 1
            else:
                mult = 1
    return f


def clamped_random_knots(rng, n_ctrl: int, p: int, repeat_prob: float = 0.0):
    inner = _interior_knots(rng, n_ctrl - p - 1, p, repeat_prob)
    return np.concatenate([np.zeros(p + 1, np.float32), inner,
                           np.ones(p + 1, np.float32)]).astype(np.float32)


def perturbed_lattice(rng, nu_c: int, nv_c: int, jitter: float = 0.3,
                      zamp: float = 0.2) -> np.ndarray:
    """x = i/(nu_c-1) + U(-j,j)/(nu_c-1), y likewise in j, z ~ U(-zamp, zamp)."""
    i = np.arange(nu_c, dtype=np.float64)[:, None] * np.ones((1, nv_c))
    j = np.ones((nu_c, 1)) * np.arange(nv_c, dtype=np.float64)[None, :]
    du = max(nu_c - 1, 1)
    dv = max(nv_c - 1, 1)
    x = (i + rng.uniform(-jitter, jitter, (nu_c, nv_c))) / du
    y = (j + rng.uniform(-jitter, jitter, (nu_c, nv_c))) / dv
    z = rng.uniform(-zamp, zamp, (nu_c, nv_c))
    return np.stack([x, y, z], axis=-1).astype(np.float32)


def _grid_target(rng, us, vs, zamp=0.2):
    uu, vv = np.meshgrid(us.astype(np.float64), vs.astype(np.float64), indexing="ij")
    z = rng.uniform(-zamp, zamp, uu.shape)
    return np.stack([uu, vv, z], axis=-1).astype(np.float32)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def single_bicubic(seed: int = 0) -> Batch:
    """One bicubic 8x8 surface, lattice P_ij = (i/7, j/7, z), 64x64 samples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = q = 3
    nc = 8
    i = np.arange(nc, dtype=np.float64)
    ctrl = np.zeros((nc, nc, 3))
    ctrl[..., 0] = i[:, None] / 7.0
    ctrl[..., 1] = i[None, :] / 7.0
    ctrl[..., 2] = rng.uniform(-0.2, 0.2, (nc, nc))
    w = rng.uniform(0.5, 1.5, (nc, nc))
    k = np.array([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], np.float64)
    us = uniform_grid(64)
    d = dict(p=p, q=q, nu_c=nc, nv_c=nc, nu_s=64, nv_s=64,
             ctrl=ctrl.astype(np.float32), w=w.astype(np.float32),
             ku=k.astype(np.float32), kv=k.astype(np.float32), us=us, vs=us.copy())
    d["target"] = _grid_target(rng, us, us)
    return pack("single_bicubic_8x8_64x64", [d])


def batch_bicubic(seed: int = 1, n_surf: int = 256, nc: int = 16, ns: int = 128) -> Batch:
    """256 bicubic 16x16 surfaces, 12 random interior knots, 128x128 samples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = q = 3
    us = uniform_grid(ns)
    parts = []
    for _ in range(n_surf):
        d = dict(p=p, q=q, nu_c=nc, nv_c=nc, nu_s=ns, nv_s=ns)
        d["ctrl"] = perturbed_lattice(rng, nc, nc)
        d["w"] = rng.uniform(0.5, 1.5, (nc, nc)).astype(np.float32)
        d["ku"] = clamped_random_knots(rng, nc, p)
        d["kv"] = clamped_random_knots(rng, nc, q)
        d["us"], d["vs"] = us, us
        d["target"] = _grid_target(rng, us, us)
        parts.append(d)
    return pack(f"batch_bicubic_{n_surf}x{nc}x{nc}_{ns}x{ns}", parts)


def fit_target(seed: int = 2, nc: int = 64, ns: int = 512) -> Batch:
    """Flat 64x64 bicubic initial net and samples of z = sin(3x) cos(3y)."""
    p = q = 3
    i = np.arange(nc, dtype=np.float64) / (nc - 1)
    ctrl = np.zeros((nc, nc, 3))
    ctrl[..., 0] = i[:, None]
    ctrl[..., 1] = i[None, :]
    us = uniform_grid(ns)
    x = us.astype(np.float64)
    xx, yy = np.meshgrid(x, x, indexing="ij")
    tgt = np.stack([xx, yy, np.sin(3 * xx) * np.cos(3 * yy)], -1)
    d = dict(p=p, q=q, nu_c=nc, nv_c=nc, nu_s=ns, nv_s=ns,
             ctrl=ctrl.astype(np.float32), w=np.ones((nc, nc), np.float32),
             ku=clamped_uniform_knots(nc, p), kv=clamped_uniform_knots(nc, q),
             us=us, vs=us.copy(), target=tgt.astype(np.float32))
    return pack(f"fit_{nc}x{nc}_{ns}x{ns}", [d])


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def uneven_batch(seed: int = 3, n_surf: int = 4096, with_upstream: bool = True,
                 repeat_prob: float = 0.1) -> Batch:
    """4096 surfaces of uneven degree, control-net and sample-grid size.

    p, q ~ U{1..5}; control sides round(exp(U(ln 4, ln 48))) raised to >= p+1;
    sample sides round(exp(U(ln 16, ln 256))); interior knots sorted U(0,1)
    with 10% repeats (multiplicity <= degree); perturbed-lattice nets;
    weights U(0.5, 1.5).  The upstream gradient dL/dS ~ U(-0.1, 0.1) stands in
    for 2(S - T) with T = S + U(-0.05, 0.05).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _ in range(n_surf):
        p = int(rng.integers(1, 6))
        q = int(rng.integers(1, 6))
        nu_c = max(_log_uniform_int(rng, 4, 48), p + 1)
        nv_c = max(_log_uniform_int(rng, 4, 48), q + 1)
        nu_s = _log_uniform_int(rng, 16, 256)
        nv_s = _log_uniform_int(rng, 16, 256)
        d = dict(p=p, q=q, nu_c=nu_c, nv_c=nv_c, nu_s=nu_s, nv_s=nv_s)
        d["ctrl"] = perturbed_lattice(rng, nu_c, nv_c)
        d["w"] = rng.uniform(0.5, 1.5, (nu_c, nv_c)).astype(np.float32)
        d["ku"] = clamped_random_knots(rng, nu_c, p, repeat_prob)
        d["kv"] = clamped_random_knots(rng, nv_c, q, repeat_prob)
        d["us"] = uniform_grid(nu_s)
        d["vs"] = uniform_grid(nv_s)
        parts.append(d)
    b = pack(f"uneven_batch_{n_surf}", parts)
    if with_upstream:
        b.upstream = rng.uniform(-0.1, 0.1, b.n_pts_floats).astype(np.float32)
    return b


# --------------------------------------------------------------------------
# curves
# --------------------------------------------------------------------------

@dataclasses.dataclass
class CurveBatch:
    """B rational B-spline curves of one shape (float32 inputs):
    ``ctrl [B][nc][dim]``, ``w [B][nc]``, ``knots [B][nc+p+1]``, ``us [ns]``
    (shared) or ``[B][ns]``, ``upstream [B][ns][dim]`` (dL/dC)."""

    name: str
    p: int
    nc: int
    ns: int
    dim: int
    ctrl: np.ndarray
    w: np.ndarray
    knots: np.ndarray
    us: np.ndarray
    upstream: np.ndarray

    @property
    def B(self) -> int:
        return int(self.ctrl.shape[0])

    @property
    def n_points(self) -> int:
        return self.B * self.ns


def curve_batch(seed: int = 5, B: int = 64, p: int = 3, nc: int = 16, ns: int = 256, dim: int = 3,
                repeat: float = 0.1, shared_u: bool = True, shuffle: bool = False) -> CurveBatch:
    """Curves in the plane or in space, standing in for the curve fits of the
    paper's curve-fitting section: control polygons along a jittered circle
    (x = cos t + U(-0.2, 0.2), y = sin t + U(-0.2, 0.2), z ~ U(-0.3, 0.3)),
    weights U(0.5, 1.5), clamped knots with sorted U(0,1) interior knots and
    ``repeat`` repeated ones (multiplicity <= p).  Parameters: the uniform
    grid a/(ns-1) shared by all curves, or per curve ns sorted U(0,1) draws
    (``shared_u=False``), optionally in random order (``shuffle``).
    dL/dC ~ U(-0.1, 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.linspace(0.0, 2.0 * math.pi, nc, endpoint=False)[None, :] + rng.uniform(0, 2 * math.pi, (B, 1))
    ctrl = np.zeros((B, nc, dim))
    ctrl[..., 0] = np.cos(t) + rng.uniform(-0.2, 0.2, (B, nc))
    ctrl[..., 1] = np.sin(t) + rng.uniform(-0.2, 0.2, (B, nc))
    if dim == 3:
        ctrl[..., 2] = rng.uniform(-0.3, 0.3, (B, nc))
    w = rng.uniform(0.5, 1.5, (B, nc))
    knots = np.stack([clamped_random_knots(rng, nc, p, repeat) for _ in range(B)])
    if shared_u and not shuffle:
        us = uniform_grid(ns)
    else:
        us = np.sort(rng.uniform(0.0, 1.0, (B, ns)), axis=1).astype(np.float32)
        if shuffle:
            us = np.stack([us[c][rng.permutation(ns)] for c in range(B)])
    up = rng.uniform(-0.1, 0.1, (B, ns, dim)).astype(np.float32)
    return CurveBatch(name=f"curves_{B}x{nc}_p{p}_{ns}_d{dim}", p=p, nc=nc, ns=ns, dim=dim,
                      ctrl=ctrl.astype(np.float32), w=w.astype(np.float32), knots=knots, us=us, upstream=up)


# --------------------------------------------------------------------------
# surfaces at scattered (u, v) pairs
# --------------------------------------------------------------------------

@dataclasses.dataclass
class UvBatch:
    """B surfaces of one shape and their scattered parameter pairs:
    ``ctrl [B][nu_c][nv_c][3]``, ``w [B][nu_c][nv_c]``, ``ku [B][nu_c+p+1]``,
    ``kv [B][nv_c+q+1]``, ``uv [npts][2]`` (shared) or ``[B][npts][2]``,
    ``upstream [B][npts][3]`` (dL/dS)."""

    name: str
    p: int
    q: int
    ctrl: np.ndarray
    w: np.ndarray
    ku: np.ndarray
    kv: np.ndarray
    uv: np.ndarray
    upstream: np.ndarray

    @property
    def B(self) -> int:
        return int(self.ctrl.shape[0])

    @property
    def npts(self) -> int:
        return int(self.uv.shape[-2])


def uv_batch(seed: int = 7, B: int = 4, p: int = 3, q: int = 3, nu_c: int = 16, nv_c: int = 16,
             npts: int = 4096, repeat: float = 0.1, shared_uv: bool = False) -> UvBatch:
    """Perturbed-lattice nets (as the grids), weights U(0.5, 1.5), clamped
    random knots with ``repeat`` repeated interior knots, and npts pairs
    drawn U(0,1)^2 in random order -- the parameters a point cloud carries
    (the paper's point-cloud fits).  dL/dS ~ U(-0.1, 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ctrl = np.stack([perturbed_lattice(rng, nu_c, nv_c) for _ in range(B)])
    w = rng.uniform(0.5, 1.5, (B, nu_c, nv_c)).astype(np.float32)
    ku = np.stack([clamped_random_knots(rng, nu_c, p, repeat) for _ in range(B)])
    kv = np.stack([clamped_random_knots(rng, nv_c, q, repeat) for _ in range(B)])
    shape = (npts, 2) if shared_uv else (B, npts, 2)
    uv = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    up = rng.uniform(-0.1, 0.1, (B, npts, 3)).astype(np.float32)
    return UvBatch(name=f"uv_{B}x{nu_c}x{nv_c}_p{p}q{q}_{npts}", p=p, q=q, ctrl=ctrl, w=w, ku=ku, kv=kv, uv=uv,
                   upstream=up)


# --------------------------------------------------------------------------
# point sets for the Chamfer / Hausdorff losses
# --------------------------------------------------------------------------

def point_sets(seed: int = 6, B: int = 1, n: int = 16384, m: int = 16384, dim: int = 3,
               lattice: bool = False):
    """B pairs (P [B][n][dim], Q [B][m][dim]) standing in for evaluated
    surface points and a scanned target cloud: P on the unit square at
    uniform random (u, v) with z = 0.2 sin(3u) cos(3v), Q the same surface at
    other random parameters with U(-0.02, 0.02) noise.  With ``lattice``,
    both are points of the integer lattice {0..7}^dim scaled by 1/8, so
    many squared distances tie exactly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if lattice:
        P = rng.integers(0, 8, (B, n, dim)) / 8.0
        Q = rng.integers(0, 8, (B, m, dim)) / 8.0
        return P.astype(np.float32), Q.astype(np.float32)

    def draw(k, noise):
        u = rng.uniform(0.0, 1.0, (B, k))
        v = rng.uniform(0.0, 1.0, (B, k))
        X = np.stack([u, v, 0.2 * np.sin(3 * u) * np.cos(3 * v)], -1)[..., :dim]
        return X + rng.uniform(-noise, noise, X.shape)

    return draw(n, 0.0).astype(np.float32), draw(m, 0.02).astype(np.float32)


WORKLOADS = {
    "single_bicubic": single_bicubic,
    "batch_bicubic": batch_bicubic,
    "fit_target": fit_target,
    "uneven_batch": uneven_batch,
}
