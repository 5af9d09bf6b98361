"""The named synthetic workloads.

Each builder returns a :class:`Problem`: grid levels with their raw signed
distances (float32), an optional band threshold that restricts a level's
training points to ``|S| < band``, and packed float32 initial parameters.

Workloads (seed in brackets):

* tiny [0]: sphere r=0.5 on 32^3; 64 kernels with centres uniform in volume
  in the shell 0.4 < |c| < 0.6; log-scales ln 8 +- 0.1; cull factor 3.
* mid [1]: smooth union (k=0.05) of 8 ellipsoids (semi-axes U[0.1,0.4],
  random rotations) on 128^3; 2048 kernels from points with |S| < 0.05;
  log-scales U[ln 4, ln 16].
* large [2]: smooth union of 12 boxes, 6 capsules and 4 tori on levels
  64^3 -> 128^3 -> 256^3 (the finest restricted to |S| < 0.1); 1024 initial
  kernels with log-scales U[ln 16, ln 64].  The timing snapshot draws 16384
  kernels with the same rule on the three-level set.
* batching [3, shape b uses 1000+b]: 64 shapes, grids from
  {32,48,64,96,128}^3, kernel counts U[256,4096], 2-10 ellipsoids/tori.
* diff [4]: smooth union of 32 primitives (8 each of ellipsoid, box, capsule,
  torus) on 512^3 with 65536 kernels, log-scales U[ln 32, ln 128].
"""

from dataclasses import dataclass, field
from typing import List, Optional

import os

import numpy as np

from .grid import axis_coords, grid_points
from .params import random_euler_angles, init_params_from_points, init_params_in_shell, pack_params
from .sdf import random_shape, sample_sdf, sphere, surface_samples

LN = np.log


@dataclass
class LevelData:
    n: int
    axis: np.ndarray            # float32 (n,)
    S: np.ndarray               # float32 (n^3,) raw signed distance, x fastest
    band: Optional[float] = None  # training points restricted to |S| < band
    octree: bool = False        # training points: the octree layer below the previous level
    samples: Optional[np.ndarray] = None  # a surface-sample level: float32 (K, 3) points of P
    sample_cap: int = 0         # its index slots (>= K); n is then its binning grid

    @property
    def npts(self) -> int:
        return self.sample_cap if self.samples is not None else self.n ** 3

    def active_mask(self) -> Optional[np.ndarray]:
        if self.samples is not None:
            raise ValueError("a sample level has no grid mask")
        if self.octree:
            raise ValueError("an octree level's points follow from its parent level; the library and the "
                             "oracle each build them")
        if self.band is None:
            return None
        return np.abs(self.S.astype(np.float64)) < self.band


@dataclass
class Problem:
    name: str
    levels: List[LevelData]
    params: np.ndarray          # packed float32, 11 * cap
    m: int
    cap: int
    cull_k: float = 3.0
    weight_map: int = 0         # 0: a = w|w| ; 1: a = w
    orientation: int = 0        # 0: quaternion ; 1: Euler angles in the first three q slots
    lr: float = 1e-3
    lam: float = 1e-4
    steps: int = 1
    extra: dict = field(default_factory=dict)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def make_tiny(seed: int = 0, n: int = 32, m: int = 64) -> Problem:
    rng = _rng(seed)
    ax = axis_coords(n)
    S = sample_sdf([sphere(0.5)], ax)
    w, c, s, q = init_params_in_shell(m, 0.4, 0.6, (LN(8) - 0.1, LN(8) + 0.1), rng)
    return Problem("tiny", [LevelData(n, ax, S)], pack_params(w, c, s, q), m, m,
                   cull_k=3.0, lr=1e-3, lam=1e-4, steps=100)


def make_mid(seed: int = 1, n: int = 128, m: int = 2048) -> Problem:
    rng = _rng(seed)
    prims = random_shape(["ellipsoid"] * 8, rng)
    ax = axis_coords(n)
    S = sample_sdf(prims, ax)
    w, c, s, q = init_params_from_points(grid_points(ax), S, m, (LN(4), LN(16)), rng)
    return Problem("mid", [LevelData(n, ax, S)], pack_params(w, c, s, q), m, m,
                   cull_k=3.0, lr=1e-2, steps=500, extra={"prims": prims})


def _large_shape(rng):
    return random_shape(["box"] * 12 + ["capsule"] * 6 + ["torus"] * 4, rng)


def _levels(prims, ns, bands, octree=None):
    out = []
    octree = octree or [False] * len(ns)
    for li, (n, b, o) in enumerate(zip(ns, bands, octree)):
        if o and (li == 0 or ns[li - 1] * 2 != n or b is not None):
            raise ValueError("an octree level doubles the previous level and has no band")
        ax = axis_coords(n)
        out.append(LevelData(n, ax, sample_sdf(prims, ax), b, bool(o)))
    return out


def _union_points(levels):
    pts, sd = [], []
    for lv in levels:
        if lv.samples is not None:
            continue
        p = grid_points(lv.axis)
        act = None if lv.octree else lv.active_mask()
        if act is not None:
            p, s_ = p[act], lv.S[act]
        else:
            s_ = lv.S
        pts.append(p)
        sd.append(s_)
    return np.concatenate(pts), np.concatenate(sd)


def make_large(seed: int = 2, ns=(64, 128, 256), m0: int = 1024, cap: int = 16384) -> Problem:
    rng = _rng(seed)
    prims = _large_shape(rng)
    levels = _levels(prims, ns, [None] * (len(ns) - 1) + [0.1])
    pts = grid_points(levels[0].axis)
    w, c, s, q = init_params_from_points(pts, levels[0].S, m0, (LN(16), LN(64)), rng)
    return Problem("large", levels, pack_params(w, c, s, q, cap), m0, cap, cull_k=3.0,
                   lr=1e-2, steps=1000, extra={"prims": prims})


def make_large_snapshot(seed: int = 2, ns=(64, 128, 256), m: int = 16384, octree: bool = False,
                        samples: int = 0, sample_bins: int = 64) -> Problem:
    """Timing snapshot of the large hierarchy: all three levels active and
    ``m`` kernels drawn with the init rule over the union of their points.
    ``octree`` makes the finer levels octree layers (in place of the band of
    the finest); ``samples`` > 0 appends that many surface samples binned on
    ``sample_bins`` cells per axis."""
    rng = _rng(seed)
    prims = _large_shape(rng)
    if octree:
        levels = _levels(prims, ns, [None] * len(ns), [False] + [True] * (len(ns) - 1))
    else:
        levels = _levels(prims, ns, [None] * (len(ns) - 1) + [0.1])
    pts, sd = _union_points(levels)
    w, c, s, q = init_params_from_points(pts, sd, m, (LN(16), LN(64)), rng)
    if samples > 0:
        P = surface_samples(prims, samples, _rng(seed + 7919))
        levels.append(LevelData(int(sample_bins), None, None, None, False, P, int(samples)))
    return Problem("large_snapshot", levels, pack_params(w, c, s, q), m, m, cull_k=3.0,
                   lr=1e-2, steps=1000, extra={"prims": prims})


def make_batching(seed: int = 3, shapes: int = 64, sizes=(32, 48, 64, 96, 128),
                  m_range=(256, 4096)) -> List[Problem]:
    rng = _rng(seed)
    out = []
    lams = (1e-5, 1e-4, 1e-3)
    for b in range(shapes):
        n = int(rng.choice(sizes))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        lam = float(rng.choice(lams))
        srng = _rng(1000 + b)
        k = int(srng.integers(2, 11))
        kinds = ["ellipsoid" if srng.random() < 0.5 else "torus" for _ in range(k)]
        prims = random_shape(kinds, srng)
        ax = axis_coords(n)
        S = sample_sdf(prims, ax)
        band = 0.05
        while np.count_nonzero(np.abs(S) < band) < m:
            band *= 1.5
        w, c, s, q = init_params_from_points(grid_points(ax), S, m, (LN(4), LN(16)), srng, band=band)
        out.append(Problem(f"batch{b}", [LevelData(n, ax, S)], pack_params(w, c, s, q), m, m,
                           cull_k=3.0, lr=1e-3, lam=lam, steps=200, extra={"prims": prims}))
    return out


def make_diff(seed: int = 4, n: int = 512, m: int = 65536) -> Problem:
    rng = _rng(seed)
    prims = random_shape(["ellipsoid"] * 8 + ["box"] * 8 + ["capsule"] * 8 + ["torus"] * 8, rng)
    ax = axis_coords(n)
    S = sample_sdf(prims, ax)
    w, c, s, q = init_params_from_points(grid_points(ax), S, m, (LN(32), LN(128)), rng)
    return Problem("diff", [LevelData(n, ax, S)], pack_params(w, c, s, q), m, m, cull_k=3.0,
                   lr=1e-2, steps=2000, extra={"prims": prims})


def make_custom(seed: int, ns, m: int, log_scale_range, kinds=("ellipsoid",) * 4,
                bands=None, cap: int = None, cull_k: float = 3.0, weight_map: int = 0,
                center_band: float = 0.05, orientation: int = 0, octree=None, samples=None) -> Problem:
    """Small problems for tests: any level list, any kernel count."""
    rng = _rng(seed)
    prims = random_shape(list(kinds), rng)
    bands = bands or [None] * len(ns)
    levels = _levels(prims, ns, bands, octree)
    if samples is not None:
        # (position in the level list, sample count, binning cells per axis, capacity or None)
        at, count, nbin = samples[:3]
        cap_s = samples[3] if len(samples) > 3 and samples[3] is not None else count
        P = surface_samples(prims, count, _rng(seed + 7919))
        levels.insert(at, LevelData(int(nbin), None, None, None, False, P, int(cap_s)))
    pts, sd = _union_points(levels)
    band = center_band
    while np.count_nonzero(np.abs(sd) < band) < m:
        band *= 1.5
    w, c, s, q = init_params_from_points(pts, sd, m, log_scale_range, rng, band=band)
    if orientation == 1:
        q = random_euler_angles(m, rng)
    cap = m if cap is None else cap
    return Problem(f"custom{seed}", levels, pack_params(w, c, s, q, cap), m, cap,
                   cull_k=cull_k, weight_map=weight_map, orientation=orientation, extra={"prims": prims})


def save_problem(prob: Problem, path: str) -> None:
    """Write a problem's arrays and settings to an npz file (no pickles; the
    primitives in `extra` are not kept)."""
    arrs = {"params": prob.params,
            "meta": np.array([prob.m, prob.cap, prob.weight_map, prob.orientation, prob.steps, len(prob.levels)],
                             np.int64),
            "fmeta": np.array([prob.cull_k, prob.lr, prob.lam], np.float64),
            "name": np.array(prob.name)}
    for i, lv in enumerate(prob.levels):
        if lv.axis is not None:
            arrs[f"l{i}_axis"] = lv.axis
            arrs[f"l{i}_S"] = lv.S
        arrs[f"l{i}_meta"] = np.array([lv.n, lv.band is not None, lv.band or 0.0, lv.octree,
                                       lv.samples is not None, lv.sample_cap], np.float64)
        if lv.samples is not None:
            arrs[f"l{i}_samples"] = lv.samples
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def load_problem(path: str) -> Problem:
    with np.load(path, allow_pickle=False) as z:
        m, cap, wm, orient, steps, nl = (int(v) for v in z["meta"])
        cull_k, lr, lam = (float(v) for v in z["fmeta"])
        levels = []
        for i in range(nl):
            n, has_band, band, octree, has_samples, scap = z[f"l{i}_meta"]
            grid = f"l{i}_axis" in z.files
            levels.append(LevelData(int(n), z[f"l{i}_axis"] if grid else None, z[f"l{i}_S"] if grid else None,
                                    float(band) if has_band else None,
                                    bool(octree), z[f"l{i}_samples"] if has_samples else None, int(scap)))
        return Problem(str(z["name"]), levels, z["params"], m, cap, cull_k, wm, orient, lr, lam, steps)
