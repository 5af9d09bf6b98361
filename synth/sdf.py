"""Analytic signed distance fields used as synthetic training data.

The distances are textbook formulas, evaluated in float64 in each
primitive's local frame and stored as float32:

* sphere    ``|p| - r``
* ellipsoid ``min(a) * (|p / a| - 1)`` (a 1-Lipschitz bound with the exact zero set)
* box       ``|max(|p| - b, 0)| + min(max_k(|p_k| - b_k), 0)``
* capsule   distance to the segment ``[(-L/2,0,0), (L/2,0,0)]`` minus ``r``
* torus     ``|(|p_xy| - R, p_z)| - r``

Shapes combine primitives with the polynomial smooth minimum
``smin_k(a, b) = min(a, b) - max(k - |a - b|, 0)^2 / (4 k)``, folded left in
generation order.  Rotations of primitives are Haar-random orthogonal
matrices (QR of a Gaussian matrix with the sign fix) with determinant +1.
"""

import os
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np


@dataclass
class Primitive:
    kind: str                      # sphere | ellipsoid | box | capsule | torus
    center: np.ndarray             # (3,) float64
    rot: np.ndarray                # (3, 3) local -> world rotation
    params: Sequence[float] = field(default_factory=tuple)

    def local(self, p: np.ndarray) -> np.ndarray:
        # world point -> local frame: rot^T (p - center), for row-vector p
        # (written out elementwise so that no threaded BLAS call is involved)
        d = p - self.center
        r = self.rot
        return d[:, 0:1] * r[0] + d[:, 1:2] * r[1] + d[:, 2:3] * r[2]

    def distance(self, p: np.ndarray) -> np.ndarray:
        q = self.local(p)
        k = self.kind
        if k == "sphere":
            (r,) = self.params
            return np.linalg.norm(q, axis=1) - r
        if k == "ellipsoid":
            a = np.asarray(self.params, dtype=np.float64)
            return a.min() * (np.linalg.norm(q / a, axis=1) - 1.0)
        if k == "box":
            b = np.asarray(self.params, dtype=np.float64)
            d = np.abs(q) - b
            outside = np.linalg.norm(np.maximum(d, 0.0), axis=1)
            inside = np.minimum(d.max(axis=1), 0.0)
            return outside + inside
        if k == "capsule":
            length, r = self.params
            x = np.clip(q[:, 0], -0.5 * length, 0.5 * length)
            dx = q[:, 0] - x
            return np.sqrt(dx * dx + q[:, 1] ** 2 + q[:, 2] ** 2) - r
        if k == "torus":
            big, small = self.params
            rho = np.sqrt(q[:, 0] ** 2 + q[:, 1] ** 2) - big
            return np.sqrt(rho * rho + q[:, 2] ** 2) - small
        raise ValueError(f"unknown primitive {k!r}")


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((3, 3))
    qm, rm = np.linalg.qr(g)
    qm = qm * np.sign(np.diag(rm))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def sphere(r: float, center=(0.0, 0.0, 0.0)) -> Primitive:
    return Primitive("sphere", np.asarray(center, np.float64), np.eye(3), (float(r),))


def ellipsoid(semi_axes, center, rot) -> Primitive:
    return Primitive("ellipsoid", np.asarray(center, np.float64), np.asarray(rot, np.float64),
                     tuple(float(a) for a in semi_axes))


def box(half_extents, center, rot) -> Primitive:
    return Primitive("box", np.asarray(center, np.float64), np.asarray(rot, np.float64),
                     tuple(float(b) for b in half_extents))


def capsule(length, radius, center, rot) -> Primitive:
    return Primitive("capsule", np.asarray(center, np.float64), np.asarray(rot, np.float64),
                     (float(length), float(radius)))


def torus(big, small, center, rot) -> Primitive:
    return Primitive("torus", np.asarray(center, np.float64), np.asarray(rot, np.float64),
                     (float(big), float(small)))


def random_primitive(kind: str, rng: np.random.Generator) -> Primitive:
    """One primitive with the default placement ranges."""
    c = rng.uniform(-0.5, 0.5, size=3)
    rot = _haar_rotation(rng)
    if kind == "ellipsoid":
        return ellipsoid(rng.uniform(0.1, 0.4, size=3), c, rot)
    if kind == "box":
        return box(rng.uniform(0.05, 0.3, size=3), c, rot)
    if kind == "capsule":
        return capsule(rng.uniform(0.2, 0.6), rng.uniform(0.03, 0.1), c, rot)
    if kind == "torus":
        return torus(rng.uniform(0.15, 0.35), rng.uniform(0.03, 0.08), c, rot)
    if kind == "sphere":
        return Primitive("sphere", c, np.eye(3), (float(rng.uniform(0.1, 0.4)),))
    raise ValueError(kind)


def random_shape(kinds: Sequence[str], rng: np.random.Generator) -> List[Primitive]:
    return [random_primitive(k, rng) for k in kinds]


def smooth_union(da: np.ndarray, db: np.ndarray, k: float) -> np.ndarray:
    h = np.maximum(k - np.abs(da - db), 0.0)
    return np.minimum(da, db) - h * h / (4.0 * k)


def _eval_points(prims: Sequence[Primitive], p: np.ndarray, k: float) -> np.ndarray:
    d = prims[0].distance(p)
    for pr in prims[1:]:
        d = smooth_union(d, pr.distance(p), k)
    return d


def surface_samples(prims: Sequence[Primitive], count: int, rng: np.random.Generator, k: float = 0.05,
                    iters: int = 12) -> np.ndarray:
    """``count`` points on the zero set of the smooth union of ``prims``
    (the surface samples P): uniform draws in [-1, 1]^3 near the surface,
    moved onto it by Newton steps along a central-difference gradient.
    Returns float32 (count, 3), inside [-1, 1]^3, |S| below 1e-5."""
    out = []
    have = 0
    e = 1e-5
    while have < count:
        p = rng.uniform(-1.0, 1.0, size=(max(4 * count, 4096), 3))
        p = p[np.abs(_eval_points(prims, p, k)) < 0.05]
        for _ in range(iters):
            d = _eval_points(prims, p, k)
            g = np.stack([(_eval_points(prims, p + e * u, k) - _eval_points(prims, p - e * u, k)) / (2 * e)
                          for u in np.eye(3)], axis=1)
            p = p - (d / np.maximum(np.sum(g * g, axis=1), 1e-12))[:, None] * g
        p = p.astype(np.float32)
        ok = np.all(np.abs(p) <= 1.0, axis=1) & (np.abs(_eval_points(prims, p.astype(np.float64), k)) < 1e-5)
        out.append(p[ok])
        have += int(ok.sum())
    return np.concatenate(out)[:count]


def _eval_slabs(prims, a, k, z0, z1):
    n = a.size
    yy, xx = np.meshgrid(a, a, indexing="ij")
    xy = np.stack([xx.ravel(), yy.ravel()], axis=1)
    plane = n * n
    out = np.empty((z1 - z0) * plane, dtype=np.float32)
    for zs in range(z0, z1, 8):
        ze = min(z1, zs + 8)
        pts = np.empty(((ze - zs) * plane, 3))
        for zi, z in enumerate(range(zs, ze)):
            pts[zi * plane:(zi + 1) * plane, :2] = xy
            pts[zi * plane:(zi + 1) * plane, 2] = a[z]
        out[(zs - z0) * plane:(ze - z0) * plane] = _eval_points(prims, pts, k).astype(np.float32)
    return out


_POOL_ARGS = None

# worker processes of sample_sdf on large grids when the caller names none
# (None: up to 16, one per host CPU); 1 keeps the sampling in this process
DEFAULT_WORKERS = None


def _pool_init(args):
    global _POOL_ARGS
    _POOL_ARGS = args


def _pool_job(span):
    prims, a, k = _POOL_ARGS
    return _eval_slabs(prims, a, k, span[0], span[1])


def sample_sdf(prims: Sequence[Primitive], axis: np.ndarray, k: float = 0.05,
               workers: int = None) -> np.ndarray:
    """Sample the smooth union of ``prims`` on the grid of ``axis``.

    Returns float32 of shape ``(n^3,)`` with x fastest.  Evaluation runs in
    float64 at the float32 grid coordinates, a few z-planes at a time; large
    grids are split over worker processes (the result does not depend
    on the split).  The workers come from multiprocessing's fork server, so
    none is a copy of a caller that has already used the GPU."""
    a = np.asarray(axis, dtype=np.float64)
    n = a.size
    if workers is None:
        workers = DEFAULT_WORKERS
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if n ** 3 >= (1 << 21) else 1
    if workers <= 1:
        return _eval_slabs(prims, a, k, 0, n)
    import multiprocessing as mp
    chunk = max(1, -(-n // (4 * workers)))
    spans = [(z, min(n, z + chunk)) for z in range(0, n, chunk)]
    with mp.get_context("forkserver").Pool(workers, initializer=_pool_init, initargs=((prims, a, k),)) as pool:
        parts = pool.map(_pool_job, spans)
    return np.concatenate(parts)
