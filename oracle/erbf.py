"""Float64 reference implementation of one SE-RBFNet optimisation step.

Test infrastructure only (see the package docstring).  Notation follows the
paper: kernel j has centre c_j, axis lengths D_j = diag(d_j1, d_j2, d_j3),
rotation R_j and weight w_j; its response at point x is

    Phi_j(x) = exp(-|| D_j R_j (x - c_j) ||^2)                 (eq. 3-7)

and the network output is

    f(x) = sum_j a_j [x in ball_j] Phi_j(x),  a_j = w_j |w_j|   (eq. 3-26, eq. 3-15-1)

Readings of the paper taken here (each also listed in the design notes):

* orientation is a unit quaternion q/|q| (Hamilton, (w, x, y, z)) by
  default; the Euler-angle form of eq. 3-6 is the alternative, read as
  R = Rz(theta_z) Ry(theta_y) Rx(theta_x) with the standard right-handed axis
  rotations (the printed Ry carries a transposed sign), and its angle
  gradients derived from dL/dR by the chain rule rather than taken from
  Appendix A;
* the optimised scale is s = ln d (per axis);
* the cull predicate is strict, ||x - c_j||^2 < r_j^2 with
  r_j = k_cull / min_k d_jk (eq. 3-15-1 with eps = exp(-k_cull^2));
* points are cell-centred grid points, several levels form one training set
  (eq. 3-16), and a level may be restricted to a band |S| < b;
* L2 is a sum over id_all (eq. 3-19), L1 the sum of |w| over kernels;
* the id_all mask is held fixed when differentiating (as in Appendix A).
"""

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Problem description consumed by the oracle
# ---------------------------------------------------------------------------


@dataclass
class OLevel:
    """One grid level: float64 copies of the float32 inputs."""
    n: int
    axis: np.ndarray                     # (n,)
    active: Optional[np.ndarray] = None  # (n^3,) bool, None = all points
    t: Optional[np.ndarray] = None       # (n^3,) targets
    S: Optional[np.ndarray] = None       # (n^3,) raw signed distance

    @property
    def npts(self):
        return self.n ** 3

    def act(self):
        return np.ones(self.npts, bool) if self.active is None else self.active


def make_level(n, axis, active=None, t=None, S=None) -> OLevel:
    f64 = lambda a: None if a is None else np.asarray(a, dtype=np.float64).reshape(-1)
    act = None if active is None else np.asarray(active, dtype=bool).reshape(-1)
    return OLevel(int(n), np.asarray(axis, dtype=np.float64), act, f64(t), f64(S))


def level_points(lv) -> np.ndarray:
    """(n^3, 3) coordinates, x fastest (the sample slots of a sample set)."""
    if isinstance(lv, OSamples):
        out = np.full((lv.cap, 3), np.nan)
        out[:lv.pts.shape[0]] = lv.pts
        return out
    a = lv.axis
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


@dataclass
class OSamples:
    """Surface samples P with label 1 (eq. 3-10 gives 1 on the surface; the
    training set of Section 3.4.2 is V = {G, P}).  `cap` index slots, the
    first K = len(pts) hold the samples (float64 copies of float32
    coordinates); `active` optionally restricts them (a mini-batch)."""
    pts: np.ndarray
    cap: int
    active: Optional[np.ndarray] = None

    @property
    def npts(self):
        return self.cap

    @property
    def t(self):
        return np.ones(self.cap)

    def act(self):
        if self.active is not None:
            return self.active
        m = np.zeros(self.cap, bool)
        m[:self.pts.shape[0]] = True
        return m


def make_samples(pts, cap=None, active=None) -> OSamples:
    p = np.asarray(pts, np.float64).reshape(-1, 3)
    return OSamples(p, p.shape[0] if cap is None else int(cap),
                    None if active is None else np.asarray(active, bool).reshape(-1))


def _sample_pairs(P: OSamples, K, j: int, radius2: Optional[float]):
    """Indices of kernel j's candidate samples (those in the ball's bounding
    box, or all) and their offsets from the centre."""
    x = P.pts
    if radius2 is None:
        idx = np.arange(x.shape[0])
    else:
        r = math.sqrt(radius2)
        inbox = np.all(np.abs(x - K.c[j][None, :]) <= r * (1 + 1e-9) + 1e-12, axis=1)
        idx = np.flatnonzero(inbox)
    d = x[idx] - K.c[j][None, :]
    return idx, d[:, 0], d[:, 1], d[:, 2]


# ---------------------------------------------------------------------------
# Targets: eq. 3-10
# ---------------------------------------------------------------------------


def sdf_min(S_levels: Sequence[np.ndarray]) -> float:
    """m = min S over every level's full grid (before any band restriction)."""
    return float(min(np.min(np.asarray(S, dtype=np.float64)) for S in S_levels))


def targets_from_sdf(S: np.ndarray, m: float) -> np.ndarray:
    """Normalised SDF of eq. 3-10: 2 exp(-h (S - m)^2) with h = ln 2 / m^2.

    Requires m < 0 (some point inside the surface)."""
    if not m < 0:
        raise ValueError("eq. 3-10 needs a negative minimum signed distance")
    S = np.asarray(S, dtype=np.float64)
    h = math.log(2.0) / (m * m)
    return 2.0 * np.exp(-h * (S - m) ** 2)


def band_mask(S: np.ndarray, band: float) -> np.ndarray:
    """Training points of a banded level: |S| < band."""
    return np.abs(np.asarray(S, dtype=np.float64)) < band


def octree_mask(S_parent: np.ndarray, n_parent: int, parent_active: Optional[np.ndarray] = None) -> np.ndarray:
    """Points of the octree layer below a level (eq. 3-16's G^i on an octree,
    read on cell-centred grids): level 2n's points are the centres of the
    eight children of each level-n cell that is subdivided.  A cell is
    subdivided when it exists (its centre is an active point of level n) and
    may meet the surface: |S(centre)| <= sqrt(3)/n, the half-diagonal of a
    cell of width 2/n (a signed distance changes by at most the distance
    moved).  Returns the (2n)^3 mask, x fastest."""
    n = int(n_parent)
    sub = np.abs(np.asarray(S_parent, np.float64).reshape(n, n, n)) <= math.sqrt(3.0) / n
    if parent_active is not None:
        sub &= np.asarray(parent_active, bool).reshape(n, n, n)
    return sub.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2).reshape(-1)


# ---------------------------------------------------------------------------
# Per-kernel quantities (eq. 3-7, eq. 3-26, eq. 3-15)
# ---------------------------------------------------------------------------


def quat_to_rot(qhat: np.ndarray) -> np.ndarray:
    """Rotation matrix of unit quaternions (w, x, y, z), shape (m, 3, 3)."""
    w, x, y, z = qhat[:, 0], qhat[:, 1], qhat[:, 2], qhat[:, 3]
    R = np.empty((qhat.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def quat_rot_jacobian(qhat: np.ndarray) -> np.ndarray:
    """dR_ab / dqhat_k of :func:`quat_to_rot`, shape (m, 4, 3, 3)."""
    w, x, y, z = qhat[:, 0], qhat[:, 1], qhat[:, 2], qhat[:, 3]
    m = qhat.shape[0]
    J = np.zeros((m, 4, 3, 3))
    o = np.zeros(m)
    J[:, 0] = np.stack([np.stack([o, -2 * z, 2 * y], -1),
                        np.stack([2 * z, o, -2 * x], -1),
                        np.stack([-2 * y, 2 * x, o], -1)], 1)
    J[:, 1] = np.stack([np.stack([o, 2 * y, 2 * z], -1),
                        np.stack([2 * y, -4 * x, -2 * w], -1),
                        np.stack([2 * z, 2 * w, -4 * x], -1)], 1)
    J[:, 2] = np.stack([np.stack([-4 * y, 2 * x, 2 * w], -1),
                        np.stack([2 * x, o, 2 * z], -1),
                        np.stack([-2 * w, 2 * z, -4 * y], -1)], 1)
    J[:, 3] = np.stack([np.stack([-4 * z, -2 * w, 2 * x], -1),
                        np.stack([2 * w, -4 * z, 2 * y], -1),
                        np.stack([2 * x, 2 * y, o], -1)], 1)
    return J


ORIENT_QUATERNION = 0
ORIENT_EULER = 1


def _axis_rotations(theta: np.ndarray):
    """Rx(tx), Ry(ty), Rz(tz) and their angle derivatives, each (m, 3, 3)."""
    m = theta.shape[0]
    out = []
    for k, t in enumerate((theta[:, 0], theta[:, 1], theta[:, 2])):
        c, s = np.cos(t), np.sin(t)
        R = np.zeros((m, 3, 3))
        dR = np.zeros((m, 3, 3))
        i, j = [(1, 2), (2, 0), (0, 1)][k]      # the plane the rotation turns
        R[:, k, k] = 1.0
        R[:, i, i] = c
        R[:, j, j] = c
        R[:, i, j] = -s
        R[:, j, i] = s
        dR[:, i, i] = -s
        dR[:, j, j] = -s
        dR[:, i, j] = -c
        dR[:, j, i] = c
        out.append((R, dR))
    return out


def euler_to_rot(theta: np.ndarray) -> np.ndarray:
    """R = Rz(theta_z) Ry(theta_y) Rx(theta_x) (eq. 3-6), shape (m, 3, 3)."""
    (Rx, _), (Ry, _), (Rz, _) = _axis_rotations(np.asarray(theta, np.float64).reshape(-1, 3))
    return Rz @ Ry @ Rx


def euler_rot_jacobian(theta: np.ndarray) -> np.ndarray:
    """dR_ab / dtheta_k of :func:`euler_to_rot`, shape (m, 3, 3, 3)."""
    (Rx, dRx), (Ry, dRy), (Rz, dRz) = _axis_rotations(np.asarray(theta, np.float64).reshape(-1, 3))
    return np.stack([Rz @ Ry @ dRx, Rz @ dRy @ Rx, dRz @ Ry @ Rx], axis=1)


@dataclass
class Kernels:
    w: np.ndarray      # (m,)
    c: np.ndarray      # (m, 3)
    s: np.ndarray      # (m, 3)
    q: np.ndarray      # (m, 4) as given
    qn: np.ndarray     # (m,) |q|
    qhat: np.ndarray   # (m, 4)
    R: np.ndarray      # (m, 3, 3)
    d: np.ndarray      # (m, 3) axis lengths exp(s)
    a: np.ndarray      # (m,) amplitude
    dadw: np.ndarray   # (m,)
    r2: np.ndarray     # (m,) squared cull radius
    weight_map: int
    orientation: int = ORIENT_QUATERNION   # q holds (theta_x, theta_y, theta_z, -) for Euler

    @property
    def m(self):
        return self.w.shape[0]


def kernels_from_packed(p: np.ndarray, m: int, cap: int, cull_k: float,
                        weight_map: int = 0, orientation: int = ORIENT_QUATERNION) -> Kernels:
    seg = np.asarray(p, dtype=np.float32).reshape(11, cap)[:, :m].astype(np.float64)
    return make_kernels(seg[0], seg[1:4].T, seg[4:7].T, seg[7:11].T, cull_k, weight_map, orientation)


def make_kernels(w, c, s, q, cull_k: float, weight_map: int = 0,
                 orientation: int = ORIENT_QUATERNION) -> Kernels:
    """Derived per-kernel quantities.

    a = w|w| (eq. 3-26) for weight_map 0, a = w for weight_map 1;
    r = k_cull / min_k d_k (eq. 3-15 with lambda_j = min_k d_jk^2);
    R from the quaternion q/|q|, or from the Euler angles q[:, :3] (eq. 3-6)."""
    w = np.asarray(w, np.float64).reshape(-1)
    c = np.asarray(c, np.float64).reshape(-1, 3)
    s = np.asarray(s, np.float64).reshape(-1, 3)
    q = np.asarray(q, np.float64).reshape(-1, 4)
    if orientation == ORIENT_EULER:
        qn = np.ones(q.shape[0])
        qhat = q.copy()
        R = euler_to_rot(q[:, :3])
    elif orientation == ORIENT_QUATERNION:
        qn = np.linalg.norm(q, axis=1)
        qhat = q / qn[:, None]
        R = quat_to_rot(qhat)
    else:
        raise ValueError("orientation must be 0 (quaternion) or 1 (Euler angles)")
    d = np.exp(s)
    if weight_map == 0:
        a = w * np.abs(w)
        dadw = 2.0 * np.abs(w)
    elif weight_map == 1:
        a = w.copy()
        dadw = np.ones_like(w)
    else:
        raise ValueError("weight_map must be 0 (signed square) or 1 (linear)")
    r = cull_k / d.min(axis=1)
    return Kernels(w, c, s, q, qn, qhat, R, d, a, dadw, r * r, weight_map, orientation)


# ---------------------------------------------------------------------------
# Forward: eq. 3-9 restricted by eq. 3-15-1
# ---------------------------------------------------------------------------


def _phi_and_u(K: Kernels, j: int, dx, dy, dz):
    """u = R_j Delta and Phi = exp(-|D_j u|^2) on broadcast offset arrays."""
    R = K.R[j]
    u = [R[k, 0] * dx + R[k, 1] * dy + R[k, 2] * dz for k in range(3)]
    e = sum((K.d[j, k] * u[k]) ** 2 for k in range(3))
    return np.exp(-e), u


def _box(axis: np.ndarray, lo: float, hi: float):
    i0 = max(0, int(np.searchsorted(axis, lo, side="left")) - 1)
    i1 = min(axis.size, int(np.searchsorted(axis, hi, side="right")) + 1)
    return i0, i1


def _kernel_box(lv: OLevel, K: Kernels, j: int, radius2: Optional[float]):
    """Index box (z, y, x ranges) holding kernel j's ball, and its offsets."""
    if radius2 is None:
        rng = [(0, lv.n)] * 3
    else:
        r = math.sqrt(radius2)
        rng = [_box(lv.axis, K.c[j, k] - r, K.c[j, k] + r) for k in range(3)]
    (x0, x1), (y0, y1), (z0, z1) = rng
    dx = (lv.axis[x0:x1] - K.c[j, 0])[None, None, :]
    dy = (lv.axis[y0:y1] - K.c[j, 1])[None, :, None]
    dz = (lv.axis[z0:z1] - K.c[j, 2])[:, None, None]
    return (z0, z1, y0, y1, x0, x1), dx, dy, dz


def forward(levels: List[OLevel], K: Kernels, culled: bool = True,
            radius_scale: Optional[np.ndarray] = None) -> List[np.ndarray]:
    """f at every point of every level (0 at inactive points).

    culled=True applies eq. 3-15-1 with the strict predicate; culled=False
    sums every kernel at every point (all pairs).  radius_scale optionally
    multiplies individual kernels' cull radii (used for finite differences)."""
    out = []
    for lv in levels:
        if isinstance(lv, OSamples):
            f = np.zeros(lv.cap)
            for j in range(K.m):
                r2 = None
                if culled:
                    r2 = K.r2[j] * (1.0 if radius_scale is None else radius_scale[j] ** 2)
                idx, dx, dy, dz = _sample_pairs(lv, K, j, r2)
                phi, _ = _phi_and_u(K, j, dx, dy, dz)
                if r2 is not None:
                    phi = np.where(dx * dx + dy * dy + dz * dz < r2, phi, 0.0)
                f[idx] += K.a[j] * phi
            out.append(np.where(lv.act(), f, 0.0))
            continue
        f = np.zeros((lv.n, lv.n, lv.n))
        for j in range(K.m):
            r2 = None
            if culled:
                r2 = K.r2[j] * (1.0 if radius_scale is None else radius_scale[j] ** 2)
            (z0, z1, y0, y1, x0, x1), dx, dy, dz = _kernel_box(lv, K, j, r2)
            phi, _ = _phi_and_u(K, j, dx, dy, dz)
            if r2 is not None:
                phi = np.where(dx * dx + dy * dy + dz * dz < r2, phi, 0.0)
            f[z0:z1, y0:y1, x0:x1] += K.a[j] * phi
        f = f.reshape(-1)
        if lv.active is not None:
            f = np.where(lv.active, f, 0.0)
        out.append(f)
    return out


def forward_at_points(pts: np.ndarray, K: Kernels, culled: bool = True) -> np.ndarray:
    """f at arbitrary points, one point at a time over all kernels (for
    sampled checks on large grids)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.empty(pts.shape[0])
    for i, x in enumerate(pts):
        delta = x[None, :] - K.c
        u = np.einsum("mkl,ml->mk", K.R, delta)
        phi = np.exp(-np.sum((K.d * u) ** 2, axis=1))
        if culled:
            phi = np.where(np.sum(delta * delta, axis=1) < K.r2, phi, 0.0)
        out[i] = np.sum(K.a * phi)
    return out


def allowance_at_points(pts: np.ndarray, K: Kernels, rel: float = 2.0 ** -20):
    """boundary_allowance (below) at arbitrary points: per point, the sum of
    |a_j| Phi over kernels whose squared distance lies within rel * r^2 of
    r^2; also the number of such pairs."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    count = 0
    for i, x in enumerate(pts):
        delta = x[None, :] - K.c
        dist2 = np.sum(delta * delta, axis=1)
        amb = np.abs(dist2 - K.r2) <= rel * K.r2
        if amb.any():
            u = np.einsum("mkl,ml->mk", K.R[amb], delta[amb])
            out[i] = np.sum(np.abs(K.a[amb]) * np.exp(-np.sum((K.d[amb] * u) ** 2, axis=1)))
            count += int(amb.sum())
    return out, count


def kernel_field(lv: OLevel, K: Kernels, j: int, radius_scale: float = 1.0):
    """One kernel's term a_j [in ball] Phi_j on its own index box (eq. 3-7,
    eq. 3-15-1, radius scaled by radius_scale): returns the box bounds
    (z0, z1, y0, y1, x0, x1) and the values, shape (z, y, x).  Used for local
    finite differences on large grids, where only this kernel's term moves."""
    r2 = K.r2[j] * radius_scale ** 2
    box, dx, dy, dz = _kernel_box(lv, K, j, r2)
    phi, _ = _phi_and_u(K, j, dx, dy, dz)
    phi = np.where(dx * dx + dy * dy + dz * dz < r2, phi, 0.0)
    return box, K.a[j] * phi


def subset(K: Kernels, idx) -> Kernels:
    """The kernels `idx` of K (their terms and gradients are independent of
    the others')."""
    idx = np.asarray(idx)
    out = Kernels(**{f: (getattr(K, f)[idx] if isinstance(getattr(K, f), np.ndarray) else getattr(K, f))
                     for f in K.__dataclass_fields__})
    return out


def truncation_bound(levels: List[OLevel], K: Kernels) -> List[np.ndarray]:
    """Per-point bound on |f_all - f_culled|: the sum over culled pairs of
    |a_j| exp(-d_min,j^2 ||Delta||^2), which dominates each dropped term."""
    out = []
    for lv in levels:
        if isinstance(lv, OSamples):
            b = np.zeros(lv.cap)
            for j in range(K.m):
                idx, dx, dy, dz = _sample_pairs(lv, K, j, None)
                dist2 = dx * dx + dy * dy + dz * dz
                b[idx] += np.where(dist2 < K.r2[j], 0.0, abs(K.a[j]) * np.exp(-K.d[j].min() ** 2 * dist2))
            out.append(b)
            continue
        b = np.zeros((lv.n, lv.n, lv.n))
        for j in range(K.m):
            (z0, z1, y0, y1, x0, x1), dx, dy, dz = _kernel_box(lv, K, j, None)
            dist2 = dx * dx + dy * dy + dz * dz
            dmin2 = K.d[j].min() ** 2
            b += np.where(dist2 < K.r2[j], 0.0, abs(K.a[j]) * np.exp(-dmin2 * dist2))
        out.append(b.reshape(-1))
    return out


def boundary_allowance(levels: List[OLevel], K: Kernels, rel: float = 2.0 ** -20):
    """Pairs whose squared distance lies within rel * r^2 of r^2: the cull
    decision there can legitimately differ between float32 and float64.
    Returns per-level arrays of sum |a_j| Phi over such pairs, and the count."""
    out, count = [], 0
    for lv in levels:
        if isinstance(lv, OSamples):
            b = np.zeros(lv.cap)
            act = lv.act()
            for j in range(K.m):
                idx, dx, dy, dz = _sample_pairs(lv, K, j, K.r2[j] * (1 + 4 * rel))
                dist2 = dx * dx + dy * dy + dz * dz
                amb = (np.abs(dist2 - K.r2[j]) <= rel * K.r2[j]) & act[idx]
                if amb.any():
                    phi, _ = _phi_and_u(K, j, dx, dy, dz)
                    b[idx] += np.where(amb, abs(K.a[j]) * phi, 0.0)
                    count += int(amb.sum())
            out.append(b)
            continue
        b = np.zeros((lv.n, lv.n, lv.n))
        for j in range(K.m):
            (z0, z1, y0, y1, x0, x1), dx, dy, dz = _kernel_box(lv, K, j, K.r2[j] * (1 + 4 * rel))
            dist2 = dx * dx + dy * dy + dz * dz
            amb = np.abs(dist2 - K.r2[j]) <= rel * K.r2[j]
            if lv.active is not None:
                amb &= lv.active.reshape(lv.n, lv.n, lv.n)[z0:z1, y0:y1, x0:x1]
            if amb.any():
                phi, _ = _phi_and_u(K, j, dx, dy, dz)
                b[z0:z1, y0:y1, x0:x1] += np.where(amb, abs(K.a[j]) * phi, 0.0)
                count += int(amb.sum())
        out.append(b.reshape(-1))
    return out, count


def pair_counts(levels: List[OLevel], K: Kernels, G: Optional[List[np.ndarray]] = None):
    """P_fwd: in-ball pairs at active points; P_bwd: those with G != 0."""
    pf = pb = 0
    for li, lv in enumerate(levels):
        if isinstance(lv, OSamples):
            act = lv.act()
            g1 = None if G is None else np.asarray(G[li])
            for j in range(K.m):
                idx, dx, dy, dz = _sample_pairs(lv, K, j, K.r2[j])
                inb = (dx * dx + dy * dy + dz * dz < K.r2[j]) & act[idx]
                pf += int(inb.sum())
                if g1 is not None:
                    pb += int((inb & (g1[idx] != 0)).sum())
            continue
        act = lv.act().reshape(lv.n, lv.n, lv.n)
        g3 = None if G is None else G[li].reshape(lv.n, lv.n, lv.n)
        for j in range(K.m):
            (z0, z1, y0, y1, x0, x1), dx, dy, dz = _kernel_box(lv, K, j, K.r2[j])
            inb = (dx * dx + dy * dy + dz * dz < K.r2[j]) & act[z0:z1, y0:y1, x0:x1]
            pf += int(inb.sum())
            if g3 is not None:
                pb += int((inb & (g3[z0:z1, y0:y1, x0:x1] != 0)).sum())
    return pf, pb


# ---------------------------------------------------------------------------
# Mask and loss: eq. 3-18, eq. 3-19, eq. 3-14_2, eq. l1_activate2
# ---------------------------------------------------------------------------


@dataclass
class LossOut:
    E: List[np.ndarray]        # residual on id_all, 0 elsewhere
    idall: List[np.ndarray]    # bool masks
    L2: float
    L1: float
    max_abs_E: float
    n_idall: int


def loss(levels: List[OLevel], f: List[np.ndarray], K: Kernels,
         tau1: float = 0.9, tau2: float = 1.1) -> LossOut:
    E_all, id_all = [], []
    L2, mx, cnt = 0.0, 0.0, 0
    for lv, fl in zip(levels, f):
        t = lv.t
        id0 = (tau1 < t) & (t < tau2)
        id1 = (t <= tau1) & (fl > tau1)
        id2 = (t >= tau2) & (fl < tau2)
        ida = (id0 | id1 | id2) & lv.act()
        E = np.where(ida, fl - t, 0.0)
        E_all.append(E)
        id_all.append(ida)
        L2 += float(np.sum(E * E))
        if ida.any():
            mx = max(mx, float(np.max(np.abs(E[ida]))))
        cnt += int(ida.sum())
    L1 = float(np.sum(np.abs(K.w)))
    return LossOut(E_all, id_all, L2, L1, mx, cnt)


def l2_frozen(levels, K, idall, culled=True, radius_scale=None):
    """L2 of eq. 3-19 with a fixed id_all (the function the gradient of
    Appendix A differentiates)."""
    f = forward(levels, K, culled=culled, radius_scale=radius_scale)
    return float(sum(np.sum(np.where(ia, fl - lv.t, 0.0) ** 2)
                     for lv, fl, ia in zip(levels, f, idall)))


# ---------------------------------------------------------------------------
# Backward: Appendix A, with the quaternion chain rule in place of angles
# ---------------------------------------------------------------------------


@dataclass
class Grads:
    w: np.ndarray   # (m,)
    c: np.ndarray   # (m, 3)
    s: np.ndarray   # (m, 3)
    q: np.ndarray   # (m, 4)
    a: np.ndarray   # (m,) dL/da

    def packed(self, cap=None):
        m = self.w.shape[0]
        cap = m if cap is None else cap
        out = np.zeros((11, cap))
        out[0, :m] = self.w
        out[1:4, :m] = self.c.T
        out[4:7, :m] = self.s.T
        out[7:11, :m] = self.q.T
        return out.reshape(-1)


def backward(levels: List[OLevel], K: Kernels, G: List[np.ndarray],
             culled: bool = True, radius_scale: Optional[np.ndarray] = None) -> Grads:
    """Gradient of sum_i G_i f_i with respect to every kernel parameter.

    For the loss L2 of eq. 3-19, G_i = 2 E_i.  With u = R (x - c):
      dL/da     = sum G Phi
      dL/dw     = dL/da * da/dw                       (Appendix A, weight)
      dL/ds_k   = -2 a d_k^2 sum G Phi u_k^2            (axis length, d = e^s)
      dL/dc     = 2 a R^T D^2 sum G Phi u               (centre)
      dL/dR_kl  = -2 a d_k^2 sum G Phi u_k Delta_l      (replaces the angles)
      dL/dq     = (I - qhat qhat^T) J^T dL/dR / |q|     (J = dR/dqhat)
    """
    m = K.m
    S0 = np.zeros(m)
    Su = np.zeros((m, 3))
    Su2 = np.zeros((m, 3))
    SuD = np.zeros((m, 3, 3))
    for lv, g in zip(levels, G):
        samples = isinstance(lv, OSamples)
        g3 = np.asarray(g, np.float64) if samples else np.asarray(g, np.float64).reshape(lv.n, lv.n, lv.n)
        for j in range(m):
            r2 = None
            if culled:
                r2 = K.r2[j] * (1.0 if radius_scale is None else radius_scale[j] ** 2)
            if samples:
                idx, dx, dy, dz = _sample_pairs(lv, K, j, r2)
                gsel = g3[idx]
            else:
                (z0, z1, y0, y1, x0, x1), dx, dy, dz = _kernel_box(lv, K, j, r2)
                gsel = g3[z0:z1, y0:y1, x0:x1]
            phi, u = _phi_and_u(K, j, dx, dy, dz)
            if r2 is not None:
                phi = np.where(dx * dx + dy * dy + dz * dz < r2, phi, 0.0)
            gp = gsel * phi
            if not gp.any():
                continue
            delta = (dx, dy, dz)
            S0[j] += gp.sum()
            for k in range(3):
                guk = gp * u[k]
                Su[j, k] += guk.sum()
                Su2[j, k] += (guk * u[k]).sum()
                for l in range(3):
                    SuD[j, k, l] += (guk * delta[l]).sum()
    a = K.a
    d2 = K.d ** 2
    gw = S0 * K.dadw
    gs = -2.0 * a[:, None] * d2 * Su2
    gc = 2.0 * a[:, None] * np.einsum("mkl,mk->ml", K.R, d2 * Su)
    gR = -2.0 * a[:, None, None] * d2[:, :, None] * SuD
    if K.orientation == ORIENT_EULER:
        # dL/dtheta_k = sum_ab dL/dR_ab dR_ab/dtheta_k; the fourth slot is unused
        gth = np.einsum("mkab,mab->mk", euler_rot_jacobian(K.q[:, :3]), gR)
        gq = np.concatenate([gth, np.zeros((m, 1))], axis=1)
    else:
        J = quat_rot_jacobian(K.qhat)
        gqhat = np.einsum("mkab,mab->mk", J, gR)
        proj = gqhat - K.qhat * np.sum(K.qhat * gqhat, axis=1, keepdims=True)
        gq = proj / K.qn[:, None]
    return Grads(gw, gc, gs, gq, S0)


# ---------------------------------------------------------------------------
# Loss weights: eq. 3-21 and the gate of eq. l1_activate2
# ---------------------------------------------------------------------------


def sign(x):
    """sign with sign(0) = 0, as the paper defines it."""
    return np.sign(np.asarray(x, np.float64))


def min_norm_alpha(g2: np.ndarray, g1: np.ndarray) -> float:
    """alpha of eq. 3-21 for dL2/dW = g2 and dL1/dW = g1, clipped to [0, 1].

    Reading: when ||g2 - g1|| = 0 every alpha gives the same direction;
    alpha = 1 is returned."""
    g1 = np.asarray(g1, np.float64)
    g2 = np.asarray(g2, np.float64)
    den = float(np.sum((g2 - g1) ** 2))
    if den == 0.0:
        return 1.0
    num = float(np.sum((g1 - g2) * g1))
    return float(min(max(num / den, 0.0), 1.0))


MODE_FIXED, MODE_DYNAMIC, MODE_L2 = 0, 1, 2


def loss_weights(mode: int, lam: float, l1_active: bool, max_abs_E: float, tau_m: float,
                 gw2: np.ndarray, w: np.ndarray):
    """(alpha, beta) for one step.

    fixed: (1, lam).  dynamic: eq. 3-21 when L1 is scheduled on and
    max|E| < tau_m, else (1, 0).  L2-only: (1, 0)."""
    if mode == MODE_FIXED:
        return 1.0, float(lam)
    if mode == MODE_DYNAMIC and l1_active and max_abs_E < tau_m:
        al = min_norm_alpha(gw2, sign(w))
        return al, 1.0 - al
    return 1.0, 0.0


def combine(gr: Grads, w: np.ndarray, alpha: float, beta: float) -> Grads:
    """alpha * dL2 + beta * dL1 (the L1 term touches only w)."""
    return Grads(alpha * gr.w + beta * sign(w), alpha * gr.c, alpha * gr.s, alpha * gr.q,
                 alpha * gr.a)


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba, with bias correction)
# ---------------------------------------------------------------------------


def adam_step(p, g, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based).  Returns new (p, m1, m2)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m1 = b1 * np.asarray(m1, np.float64) + (1 - b1) * g
    m2 = b2 * np.asarray(m2, np.float64) + (1 - b2) * g * g
    mhat = m1 / (1 - b1 ** t)
    vhat = m2 / (1 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


# ---------------------------------------------------------------------------
# Seeding new kernels: Algorithm 2 with eq. 3-22, 3-24, 3-25
# ---------------------------------------------------------------------------


@dataclass
class SeedOut:
    index: np.ndarray   # global point indices of the new kernels, in order
    w: np.ndarray
    c: np.ndarray
    s: np.ndarray
    q: np.ndarray
    n_candidates: int
    n_extreme: int


def seed(levels: List[OLevel], E: List[np.ndarray], idall: List[np.ndarray],
         top_frac: float = 0.01, k_new: int = 256, r_nms: Optional[float] = None,
         eps: float = 1e-7, min_abs_err: float = 0.0, w_rule: int = 0,
         orientation: int = ORIENT_QUATERNION, n_idall: Optional[int] = None) -> SeedOut:
    """New kernels at local extrema of |E| (Algorithm 2).

    The training set V is the grid levels plus, when registered, the surface
    samples P (OSamples entries of `levels`; Section 3.4.2, V = {G, P}).

    1. candidates: the ceil(top_frac * n_idall) grid points of id_all with the
       largest |E| (ties to the lower global index), keeping
       |E| > max(min_abs_err, eps).  n_idall counts every id_all point of V
       (default) or is given.  Samples are never candidates: a centre placed
       on a sample has distance 0 to P, and eq. 3-24 has no scale there;
    2. extreme points: a candidate survives if |E_i| >= |E_k| for every id_all
       point k of V (grid points of every level and samples) with
       ||x_k - x_i|| <= r_nms (default: twice the finest grid spacing);
    3. the first k_new survivors by (|E| desc, index asc);
    4. eq. 3-24: c = x_i; w = -sign(E)|E| (w_rule 0) or -sign(E) sqrt|E|
       (w_rule 1); d = sqrt(ln(|E| / eps)) / dbar on all axes, dbar the
       distance from x_i to the nearest registered sample of P, or |S_i|
       (the distance to the surface that P samples) when no sample is
       registered, in both cases at least the finest grid spacing h;
       orientation zero (identity quaternion, or zero Euler angles).
    Global indices run over the levels in order, x fastest inside a grid
    level, sample slots in their order inside a sample level."""
    offs = np.cumsum([0] + [lv.npts for lv in levels])
    absE = np.concatenate([np.abs(np.asarray(e, np.float64)) for e in E])
    ida = np.concatenate([np.asarray(i, bool) for i in idall])
    is_grid = np.concatenate([np.full(lv.npts, not isinstance(lv, OSamples)) for lv in levels])
    grids = [lv for lv in levels if not isinstance(lv, OSamples)]
    h_fine = min(float(lv.axis[1] - lv.axis[0]) for lv in grids)
    if r_nms is None:
        r_nms = 2.0 * h_fine
    # every registered sample (for dbar) and the id_all samples with their |E|
    # (for the extreme-point test)
    P_all, P_ida, P_absE = [], [], []
    for li, lv in enumerate(levels):
        if isinstance(lv, OSamples):
            k = lv.pts.shape[0]
            P_all.append(lv.pts)
            sel = np.flatnonzero(ida[offs[li]:offs[li] + k])
            P_ida.append(lv.pts[sel])
            P_absE.append(absE[offs[li] + sel])
    P_all = np.concatenate(P_all) if P_all else np.zeros((0, 3))
    P_ida = np.concatenate(P_ida) if P_ida else np.zeros((0, 3))
    P_absE = np.concatenate(P_absE) if P_absE else np.zeros(0)
    gid = np.flatnonzero(ida)
    if n_idall is None:
        n_idall = gid.size
    K = int(math.ceil(top_frac * n_idall))
    gcand = gid[is_grid[gid]]
    order = np.lexsort((gcand, -absE[gcand]))
    cand = gcand[order[:K]]
    cand = cand[absE[cand] > max(min_abs_err, eps)]

    def locate(g):
        li = int(np.searchsorted(offs, g, side="right") - 1)
        loc = g - offs[li]
        n = levels[li].n
        return li, loc % n, (loc // n) % n, loc // (n * n)

    def coords(g):
        li, i, j, k = locate(g)
        a = levels[li].axis
        return np.array([a[i], a[j], a[k]])

    r2 = r_nms * r_nms
    kept = []
    for g in cand:
        x = coords(g)
        ok = True
        for li, lv in enumerate(levels):
            if isinstance(lv, OSamples):
                continue
            a = lv.axis
            rng = [_box(a, x[k] - r_nms, x[k] + r_nms) for k in range(3)]
            (x0, x1), (y0, y1), (z0, z1) = rng
            dx = (a[x0:x1] - x[0])[None, None, :]
            dy = (a[y0:y1] - x[1])[None, :, None]
            dz = (a[z0:z1] - x[2])[:, None, None]
            near = dx * dx + dy * dy + dz * dz <= r2
            n = lv.n
            zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1),
                                     indexing="ij")
            gl = offs[li] + (zz * n + yy) * n + xx
            sel = near & ida[gl]
            if sel.any() and absE[g] < absE[gl[sel]].max():
                ok = False
                break
        if ok and P_ida.shape[0]:
            d = P_ida - x[None, :]
            near = np.sum(d * d, axis=1) <= r2
            if near.any() and absE[g] < P_absE[near].max():
                ok = False
        if ok:
            kept.append(g)
    kept = np.asarray(kept, dtype=np.int64)
    if kept.size:
        o2 = np.lexsort((kept, -absE[kept]))
        kept = kept[o2][:k_new]
    Eall = np.concatenate([np.asarray(e, np.float64) for e in E])
    ev = Eall[kept]
    c = np.array([coords(g) for g in kept]).reshape(-1, 3)
    if w_rule == 0:
        w = -np.sign(ev) * np.abs(ev)
    else:
        w = -np.sign(ev) * np.sqrt(np.abs(ev))
    if kept.size:
        if P_all.shape[0]:
            dist = np.array([np.sqrt(np.min(np.sum((P_all - ci[None, :]) ** 2, axis=1))) for ci in c])
        else:
            Sall = np.concatenate([np.asarray(lv.S, np.float64) if not isinstance(lv, OSamples)
                                   else np.zeros(lv.npts) for lv in levels])
            dist = np.abs(Sall[kept])
        dbar = np.maximum(dist, h_fine)
        d = np.sqrt(np.log(np.abs(ev) / eps)) / dbar
        s = np.repeat(np.log(d)[:, None], 3, axis=1)
    else:
        s = np.zeros((0, 3))
    ident = [0.0, 0.0, 0.0, 0.0] if orientation == ORIENT_EULER else [1.0, 0.0, 0.0, 0.0]
    q = np.tile(np.array(ident), (kept.size, 1))
    return SeedOut(kept, w, c, s, q, int(cand.size), int(kept.size))


# ---------------------------------------------------------------------------
# One full step, for convenience in tests
# ---------------------------------------------------------------------------


@dataclass
class StepOut:
    f: List[np.ndarray]
    loss: LossOut
    G: List[np.ndarray]
    grads_l2: Grads
    alpha: float
    beta: float
    grads: Grads
    P_fwd: int
    P_bwd: int


def step(levels: List[OLevel], K: Kernels, mode: int = MODE_FIXED, lam: float = 0.0,
         l1_active: bool = False, tau1=0.9, tau2=1.1, tau_m=0.02, culled=True,
         count_pairs=True) -> StepOut:
    f = forward(levels, K, culled=culled)
    lo = loss(levels, f, K, tau1, tau2)
    G = [2.0 * e for e in lo.E]
    gr = backward(levels, K, G, culled=culled)
    al, be = loss_weights(mode, lam, l1_active, lo.max_abs_E, tau_m, gr.w, K.w)
    pf, pb = pair_counts(levels, K, G) if count_pairs else (0, 0)
    return StepOut(f, lo, G, gr, al, be, combine(gr, K.w, al, be), pf, pb)


# ---------------------------------------------------------------------------
# Mini-batch step (Algorithm 3, inner loop over batches of B_s points)
# ---------------------------------------------------------------------------


def batch_masks(levels: List[OLevel], batch: np.ndarray) -> List[np.ndarray]:
    """Per-level boolean masks of the points of a batch given as indices into
    the concatenation of the levels' points (level order, x fastest)."""
    batch = np.asarray(batch, np.int64)
    out, base = [], 0
    for lv in levels:
        m = np.zeros(lv.npts, bool)
        sel = batch[(batch >= base) & (batch < base + lv.npts)] - base
        m[sel] = True
        out.append(m)
        base += lv.npts
    return out


def step_batch(levels: List[OLevel], K: Kernels, batch: np.ndarray, mode: int = MODE_FIXED, lam: float = 0.0,
               l1_active: bool = False, tau1=0.9, tau2=1.1, tau_m=0.02) -> StepOut:
    """One mini-batch step: the loss of eq. 3-19 and its gradient over the
    batch's points only (id_all, L2, max|E| and eq. 3-21 taken on the batch),
    with the batch a set of indices into the concatenated points."""
    bm = batch_masks(levels, batch)
    blv = [OSamples(lv.pts, lv.cap, lv.act() & m) if isinstance(lv, OSamples) else
           OLevel(lv.n, lv.axis, lv.act() & m, lv.t, lv.S) for lv, m in zip(levels, bm)]
    return step(blv, K, mode=mode, lam=lam, l1_active=l1_active, tau1=tau1, tau2=tau2, tau_m=tau_m)


# ---------------------------------------------------------------------------
# Inscribed-sphere initialisation: Algorithm 1 with eq. 3-11 / eq. 3-12
# ---------------------------------------------------------------------------


@dataclass
class InitOut:
    index: np.ndarray   # chosen points (indices into the levels' concatenated points)
    c: np.ndarray       # (M, 3) centres
    w: np.ndarray       # (M,) weights: the normalised target at the centre
    r: np.ndarray       # (M,) sphere radii
    s: np.ndarray       # (M, 3) log axis lengths from eq. 3-12 (isotropic)
    dhat: np.ndarray    # (M,) distance to the nearest other centre
    n_left: int         # candidates no sphere covers (non-zero only when m_max stopped the rounds)


def inscribed_sphere_init(levels, gamma: float = 1e-3, m_max: Optional[int] = None) -> InitOut:
    """Algorithm 1: among the interior points (1 < t < 2, eq. 3-10) of the
    active points of the grid levels in `levels`, repeatedly take the point
    farthest from the surface as a centre with weight t, and drop every point
    within that distance of it; stop when none is left (or after m_max
    centres).  The distance to the surface is the distance to the nearest
    surface sample when `levels` holds sample sets (OSamples), else |S|.
    Squared distances are ((dx^2 + dy^2) + dz^2) in float64, compared with
    r^2 (the sphere's interior and boundary).  With samples, r^2 is that
    minimum squared distance and the order of depth uses it rounded to
    float32 (ties to the lower index); without, the order uses |S|.  Then
    eq. 3-12: d = 2 sqrt(-ln(gamma / w^2)) / dhat on all three axes, dhat the
    distance to the nearest other centre (2, the domain's width, for a single
    centre), identity rotation."""
    samples = [lv for lv in levels if isinstance(lv, OSamples)]
    SP = np.concatenate([lv.pts[lv.act()[:lv.pts.shape[0]]] for lv in samples]) if samples else None
    P, T, R2, KEY = [], [], [], []
    for lv in levels:
        if isinstance(lv, OSamples):
            P.append(np.full((lv.cap, 3), np.nan))
            T.append(np.full(lv.cap, np.nan))
            R2.append(np.full(lv.cap, -1.0))
            KEY.append(np.full(lv.cap, -1.0))
            continue
        pts = level_points(lv)
        keep = lv.act() & (lv.t > 1.0) & (lv.t < 2.0)
        P.append(np.where(keep[:, None], pts, np.nan))
        T.append(np.where(keep, lv.t, np.nan))
        if SP is None:
            r = np.abs(lv.S)
            R2.append(np.where(keep, r * r, -1.0))
            KEY.append(np.where(keep, r, -1.0))
        else:
            r2 = np.full(lv.npts, -1.0)
            for i in np.flatnonzero(keep):
                d = SP - pts[i][None, :]
                r2[i] = (((d[:, 0] * d[:, 0]) + (d[:, 1] * d[:, 1])) + (d[:, 2] * d[:, 2])).min()
            R2.append(r2)
            KEY.append(np.where(keep, r2.astype(np.float32).astype(np.float64), -1.0))
    P, T, R2, KEY = np.concatenate(P), np.concatenate(T), np.concatenate(R2), np.concatenate(KEY)
    alive = KEY >= 0.0
    chosen = []
    while alive.any() and (m_max is None or len(chosen) < m_max):
        cand = np.flatnonzero(alive)
        k = int(cand[np.argmax(KEY[cand])])     # first maximum: the lowest index among ties
        chosen.append(k)
        d2 = ((P[cand, 0] - P[k, 0]) ** 2 + (P[cand, 1] - P[k, 1]) ** 2) + (P[cand, 2] - P[k, 2]) ** 2
        alive[cand[d2 <= R2[k]]] = False
    idx = np.asarray(chosen, np.int64)
    c, w, r = P[idx], T[idx], np.sqrt(R2[idx])
    M = idx.size
    if M > 1:
        dd = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
        np.fill_diagonal(dd, np.inf)
        dhat = dd.min(axis=1)
    else:
        dhat = np.full(M, 2.0)
    d = 2.0 * np.sqrt(-np.log(gamma / (w * w))) / dhat
    s = np.repeat(np.log(d)[:, None], 3, axis=1)
    return InitOut(idx, c, w, r, s, dhat, int(alive.sum()))
