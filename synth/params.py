"""Initial ERBF parameters (seeded) and the packed parameter layout.

Packed layout (float32, one buffer of ``11 * cap`` values): eleven segments of
``cap`` floats each, in the order

    w | cx cy cz | sx sy sz | qw qx qy qz

``w`` is the raw weight, ``c`` the centre, ``s`` the per-axis log-scale
(``d = exp(s)``) and ``q`` an unnormalised quaternion ``(w, x, y, z)``.
Slots at or beyond the live count ``m`` are padding.
"""

import numpy as np

PARAM_FIELDS = ("w", "cx", "cy", "cz", "sx", "sy", "sz", "qw", "qx", "qy", "qz")


def random_unit_quaternions(m: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random unit quaternions (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = rng.random(m), rng.random(m), rng.random(m)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qx = a * np.sin(2 * np.pi * u2)
    qy = a * np.cos(2 * np.pi * u2)
    qz = b * np.sin(2 * np.pi * u3)
    qw = b * np.cos(2 * np.pi * u3)
    return np.stack([qw, qx, qy, qz], axis=1)


def random_euler_angles(m: int, rng: np.random.Generator) -> np.ndarray:
    """(m, 4) orientation slots holding three angles uniform in [-pi, pi)
    and a zero fourth slot (the Euler-angle parameterisation)."""
    out = np.zeros((m, 4))
    out[:, :3] = rng.uniform(-np.pi, np.pi, size=(m, 3))
    return out


def pack_params(w, c, s, q, cap: int = None) -> np.ndarray:
    """Pack per-kernel arrays into the float32 SoA layout."""
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    m = w.size
    cap = m if cap is None else int(cap)
    if cap < m:
        raise ValueError("capacity smaller than kernel count")
    out = np.zeros((11, cap), dtype=np.float32)
    out[0, :m] = w
    out[1:4, :m] = np.asarray(c, dtype=np.float64).reshape(m, 3).T
    out[4:7, :m] = np.asarray(s, dtype=np.float64).reshape(m, 3).T
    out[7:11, :m] = np.asarray(q, dtype=np.float64).reshape(m, 4).T
    return out.reshape(-1)


def unpack_params(p: np.ndarray, m: int, cap: int = None):
    """Inverse of :func:`pack_params`: returns float32 arrays ``w, c, s, q``."""
    p = np.asarray(p)
    cap = p.size // 11 if cap is None else cap
    seg = p.reshape(11, cap)[:, :m]
    return seg[0].copy(), seg[1:4].T.copy(), seg[4:7].T.copy(), seg[7:11].T.copy()


def init_params_from_points(points: np.ndarray, sdf: np.ndarray, m: int,
                            log_scale_range, rng: np.random.Generator,
                            band: float = 0.05, w_sigma: float = 0.1):
    """Kernel init rule: centres drawn without replacement from the points with
    ``|S| < band``; ``w ~ N(0, w_sigma)``; per-axis log-scales uniform in
    ``log_scale_range``; uniform random unit quaternions."""
    cand = np.flatnonzero(np.abs(sdf) < band)
    if cand.size < m:
        raise ValueError(f"only {cand.size} near-surface points for {m} kernels")
    pick = rng.choice(cand, size=m, replace=False)
    pick.sort()
    c = points[pick]
    w = rng.normal(0.0, w_sigma, size=m)
    lo, hi = log_scale_range
    s = rng.uniform(lo, hi, size=(m, 3))
    q = random_unit_quaternions(m, rng)
    return w, c, s, q


def init_params_in_shell(m: int, r_in: float, r_out: float, log_scale_range,
                         rng: np.random.Generator, w_sigma: float = 0.1):
    """Centres uniform in volume in the shell ``r_in < |c| < r_out``."""
    v = rng.standard_normal((m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rad = np.cbrt(rng.uniform(r_in ** 3, r_out ** 3, size=m))
    c = v * rad[:, None]
    w = rng.normal(0.0, w_sigma, size=m)
    lo, hi = log_scale_range
    s = rng.uniform(lo, hi, size=(m, 3))
    q = random_unit_quaternions(m, rng)
    return w, c, s, q
