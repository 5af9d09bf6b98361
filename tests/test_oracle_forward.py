"""Pins for the oracle's targets, per-kernel quantities and forward pass.

Each test checks the oracle against something other than itself: a closed
form, a hand-derived worked example, brute force, or an invariant."""

import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --- eq. 3-10 -------------------------------------------------------------

def test_targets_golden_dyadic_values():
    for m, S, t in _read_golden("eq3_10_targets.txt"):
        got = O.targets_from_sdf(np.array([float(S)]), float(m))[0]
        assert got == pytest.approx(float(t), rel=1e-15, abs=1e-300)


def test_targets_monotone_and_range():
    S = np.linspace(-0.3, 2.0, 1001)
    t = O.targets_from_sdf(S, -0.3)
    assert np.all(np.diff(t) < 0)
    assert t[0] == pytest.approx(2.0) and np.all(t > 0) and np.all(t <= 2.0)
    # inside (S < 0) maps to (1, 2], outside to (0, 1)
    assert np.all(t[S < 0] > 1.0) and np.all(t[S > 0] < 1.0)


def test_targets_need_negative_min():
    with pytest.raises(ValueError):
        O.targets_from_sdf(np.array([0.1, 0.2]), 0.1)


# --- rotation and per-kernel quantities ----------------------------------

def test_rotation_orthonormal_and_identity():
    rng = np.random.default_rng(0)
    q = synth.random_unit_quaternions(200, rng) * rng.uniform(0.5, 3.0, size=(200, 1))
    K = O.make_kernels(np.ones(200), np.zeros((200, 3)), np.zeros((200, 3)), q, 3.0)
    I = np.eye(3)
    assert np.abs(np.einsum("mki,mkj->mij", K.R, K.R) - I).max() < 1e-14
    assert np.abs(np.linalg.det(K.R) - 1.0).max() < 1e-14
    K1 = O.make_kernels([1.0], [[0, 0, 0]], [[0, 0, 0]], [[2.5, 0, 0, 0]], 3.0)
    assert np.abs(K1.R[0] - I).max() == 0.0


def test_rotation_worked_examples():
    axes = {"x": (1, 0, 0), "y": (0, 1, 0), "z": (0, 0, 1)}
    for ax, ang, ox, oy, oz, d1, d2, d3, ex in _read_golden("rotation_worked_examples.txt"):
        half = math.radians(float(ang)) / 2
        q = [math.cos(half)] + [math.sin(half) * v for v in axes[ax]]
        d = np.array([float(d1), float(d2), float(d3)])
        c = np.array([0.1, -0.2, 0.3])
        K = O.make_kernels([1.0], [c], [np.log(d)], [q], 100.0)
        x = c + np.array([float(ox), float(oy), float(oz)])
        got = O.forward_at_points(x[None], K, culled=False)[0]
        assert got == pytest.approx(math.exp(-float(ex)), rel=1e-13)


def test_amplitude_and_radius():
    K = O.make_kernels([-0.3, 0.2], [[0, 0, 0]] * 2, [[0.0, 1.0, 2.0], [1.0, 1.0, 1.0]],
                       [[1, 0, 0, 0]] * 2, 3.0)
    assert K.a[0] == pytest.approx(-0.09) and K.a[1] == pytest.approx(0.04)
    assert K.dadw[0] == pytest.approx(0.6)
    assert K.r2[0] == pytest.approx(9.0)             # min d = e^0 = 1
    assert K.r2[1] == pytest.approx(9.0 / math.e ** 2)
    KL = O.make_kernels([-0.3], [[0, 0, 0]], [[0, 0, 0]], [[1, 0, 0, 0]], 3.0, weight_map=1)
    assert KL.a[0] == pytest.approx(-0.3) and KL.dadw[0] == 1.0


# --- forward --------------------------------------------------------------

def _tiny_level(n=16, seed=0):
    ax = synth.axis_coords(n)
    return O.make_level(n, ax)


def test_single_isotropic_kernel_closed_form():
    lv = _tiny_level(16)
    rng = np.random.default_rng(1)
    for _ in range(3):
        q = synth.random_unit_quaternions(1, rng)
        c = rng.uniform(-0.5, 0.5, size=3)
        dv = 3.0
        w = 0.7
        K = O.make_kernels([w], [c], [[math.log(dv)] * 3], q, 3.0)
        f = O.forward([lv], K, culled=False)[0]
        pts = O.level_points(lv)
        ref = w * abs(w) * np.exp(-dv * dv * np.sum((pts - c) ** 2, axis=1))
        assert np.abs(f - ref).max() < 1e-14


def test_identity_quaternion_separable_product():
    lv = _tiny_level(12)
    d = np.array([2.0, 3.5, 5.0])
    c = np.array([0.05, -0.1, 0.2])
    K = O.make_kernels([-0.5], [c], [np.log(d)], [[1, 0, 0, 0]], 3.0)
    f = O.forward([lv], K, culled=False)[0]
    pts = O.level_points(lv)
    ref = -0.25 * np.prod(np.exp(-(d ** 2) * (pts - c) ** 2), axis=1)
    assert np.abs(f - ref).max() < 1e-15


def _rand_problem(seed, n=16, m=12, lo=1.5, hi=2.5, cull=3.0):
    p = synth.make_custom(seed, [n], m, (lo, hi), kinds=("ellipsoid", "torus"))
    K = O.kernels_from_packed(p.params, p.m, p.cap, cull)
    lv = O.make_level(n, p.levels[0].axis, S=p.levels[0].S)
    return lv, K, p


def test_culled_vs_all_pairs_within_truncation_bound():
    lv, K, _ = _rand_problem(3)
    fa = O.forward([lv], K, culled=False)[0]
    fc = O.forward([lv], K, culled=True)[0]
    bound = O.truncation_bound([lv], K)[0]
    diff = np.abs(fa - fc)
    assert np.all(diff <= bound * (1 + 1e-12) + 1e-300)
    # the bound is not vacuous: something was culled
    assert bound.max() > 0 and diff.max() > 0
    # global form of the bound: e^{-k^2} sum |a_j|
    assert diff.max() <= math.exp(-9.0) * np.abs(K.a).sum()


def test_cull_predicate_brute_force_counts():
    lv, K, _ = _rand_problem(4)
    pts = O.level_points(lv)
    brute = 0
    for j in range(K.m):
        brute += int(np.sum(np.sum((pts - K.c[j]) ** 2, axis=1) < K.r2[j]))
    pf, _ = O.pair_counts([lv], K)
    assert pf == brute


def test_forward_at_points_matches_grid_forward():
    lv, K, _ = _rand_problem(5)
    f = O.forward([lv], K)[0]
    pts = O.level_points(lv)
    idx = np.random.default_rng(0).choice(pts.shape[0], 64, replace=False)
    g = O.forward_at_points(pts[idx], K)
    assert np.abs(g - f[idx]).max() < 1e-14


def _perturbed(K, **kw):
    fields = dict(w=K.w, c=K.c, s=K.s, q=K.q)
    fields.update(kw)
    return O.make_kernels(fields["w"], fields["c"], fields["s"], fields["q"],
                          3.0, K.weight_map)


def test_invariances_permutation_sign_scale_translation():
    lv, K, _ = _rand_problem(6)
    f0 = O.forward([lv], K)[0]
    perm = np.random.default_rng(0).permutation(K.m)
    Kp = O.make_kernels(K.w[perm], K.c[perm], K.s[perm], K.q[perm], 3.0)
    assert np.abs(O.forward([lv], Kp)[0] - f0).max() < 1e-13
    assert np.abs(O.forward([lv], _perturbed(K, q=-K.q))[0] - f0).max() < 1e-13
    assert np.abs(O.forward([lv], _perturbed(K, q=3.7 * K.q))[0] - f0).max() < 1e-13
    # dyadic translation of every point and centre by 2 grid spacings
    shift = 2 * (lv.axis[1] - lv.axis[0])
    lv2 = O.make_level(lv.n, lv.axis + shift)
    Kt = _perturbed(K, c=K.c + shift)
    assert np.abs(O.forward([lv2], Kt)[0] - f0).max() < 1e-13


def test_isotropic_kernels_ignore_orientation():
    lv, K, _ = _rand_problem(7)
    iso = np.repeat(K.s[:, :1], 3, axis=1)
    Ki = _perturbed(K, s=iso)
    q2 = synth.random_unit_quaternions(K.m, np.random.default_rng(9))
    f1 = O.forward([lv], Ki)[0]
    f2 = O.forward([lv], _perturbed(Ki, q=q2))[0]
    assert np.abs(f1 - f2).max() < 1e-13


def test_multi_level_and_active_mask():
    p = synth.make_custom(8, [8, 16], 10, (1.5, 2.5), bands=[None, 0.2])
    K = O.kernels_from_packed(p.params, p.m, p.cap, 3.0)
    lvs = [O.make_level(l.n, l.axis, active=l.active_mask(), S=l.S) for l in p.levels]
    f = O.forward(lvs, K)
    # level-by-level evaluation equals the joint evaluation
    assert np.array_equal(O.forward([lvs[0]], K)[0], f[0])
    act = lvs[1].active
    assert np.all(f[1][~act] == 0.0)
    full = O.forward([O.make_level(16, p.levels[1].axis)], K)[0]
    assert np.abs(f[1][act] - full[act]).max() == 0.0


def test_boundary_allowance_counts_only_near_shell():
    lv, K, _ = _rand_problem(10)
    al, cnt = O.boundary_allowance([lv], K, rel=1e-2)
    pts = O.level_points(lv)
    brute = 0
    for j in range(K.m):
        d2 = np.sum((pts - K.c[j]) ** 2, axis=1)
        brute += int(np.sum(np.abs(d2 - K.r2[j]) <= 1e-2 * K.r2[j]))
    assert cnt == brute


def test_point_evaluation_and_allowance_match_the_grid_versions():
    # forward_at_points / allowance_at_points against forward / boundary_allowance
    rng = np.random.default_rng(12)
    n = 16
    ax = (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)
    lv = O.make_level(n, ax)
    m = 9
    K = O.make_kernels(rng.normal(0, 1, m), rng.uniform(-0.6, 0.6, (m, 3)), rng.uniform(1.2, 2.2, (m, 3)),
                       rng.normal(size=(m, 4)), 3.0)
    f = O.forward([lv], K)[0]
    al, cnt = O.boundary_allowance([lv], K, rel=1e-2)
    idx = rng.choice(n ** 3, 300, replace=False)
    x = ax.astype(np.float64)
    pts = np.stack([x[idx % n], x[(idx // n) % n], x[idx // (n * n)]], axis=1)
    assert np.allclose(O.forward_at_points(pts, K), f[idx], rtol=1e-12, atol=1e-15)
    ap, _ = O.allowance_at_points(pts, K, rel=1e-2)
    assert np.allclose(ap, al[0][idx], rtol=1e-12, atol=1e-15)
    _, call = O.allowance_at_points(O.level_points(lv), K, rel=1e-2)
    assert call == cnt and cnt > 0


def _hamilton(p, q):
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_euler_rotation_is_the_quaternion_composition():
    # Rz Ry Rx equals the rotation of the Hamilton product qz * qy * qx of the
    # three axis quaternions: pins the composition order and every sign
    # against the (separately pinned) quaternion matrix
    rng = np.random.default_rng(21)
    th = rng.uniform(-math.pi, math.pi, size=(50, 3))
    R = O.euler_to_rot(th)
    for a, (tx, ty, tz) in enumerate(th):
        qx = np.array([math.cos(tx / 2), math.sin(tx / 2), 0, 0])
        qy = np.array([math.cos(ty / 2), 0, math.sin(ty / 2), 0])
        qz = np.array([math.cos(tz / 2), 0, 0, math.sin(tz / 2)])
        q = _hamilton(qz, _hamilton(qy, qx))
        assert np.abs(O.quat_to_rot(q[None])[0] - R[a]).max() < 1e-14
    assert np.abs(O.euler_to_rot(np.zeros((1, 3)))[0] - np.eye(3)).max() == 0.0


def test_euler_worked_examples():
    # the hand-derived single-axis examples, with the angle on that axis
    slot = {"x": 0, "y": 1, "z": 2}
    for ax, ang, ox, oy, oz, d1, d2, d3, ex in _read_golden("rotation_worked_examples.txt"):
        th = [0.0, 0.0, 0.0, 0.0]
        th[slot[ax]] = math.radians(float(ang))
        d = np.array([float(d1), float(d2), float(d3)])
        c = np.array([0.1, -0.2, 0.3])
        K = O.make_kernels([1.0], [c], [np.log(d)], [th], 100.0, orientation=O.ORIENT_EULER)
        x = c + np.array([float(ox), float(oy), float(oz)])
        got = O.forward_at_points(x[None], K, culled=False)[0]
        assert got == pytest.approx(math.exp(-float(ex)), rel=1e-13)


def test_euler_jacobian_matches_differences():
    rng = np.random.default_rng(22)
    th = rng.uniform(-3, 3, size=(20, 3))
    J = O.euler_rot_jacobian(th)
    h = 1e-6
    for k in range(3):
        tp, tm = th.copy(), th.copy()
        tp[:, k] += h
        tm[:, k] -= h
        fd = (O.euler_to_rot(tp) - O.euler_to_rot(tm)) / (2 * h)
        assert np.abs(fd - J[:, k]).max() < 1e-9


def _sphere_level(n, radius=0.5):
    ax = (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)
    z, y, x = np.meshgrid(ax.astype(np.float64), ax, ax, indexing="ij")
    S = (np.sqrt(x * x + y * y + z * z) - radius).astype(np.float32).reshape(-1)
    m = O.sdf_min([S])
    t = O.targets_from_sdf(S, m).astype(np.float32)
    return O.make_level(n, ax, t=t, S=S)


def test_inscribed_sphere_init_greedy_properties():
    lv = _sphere_level(24)
    out = O.inscribed_sphere_init([lv])
    pts = O.level_points(lv)
    interior = (lv.t > 1) & (lv.t < 2)
    # the first sphere sits where |S| is largest (the grid points nearest the
    # centre), with the largest target
    assert out.r[0] == np.abs(lv.S[interior]).max() and out.w[0] == lv.t[out.index[0]]
    # greedy order: radii do not increase; each centre lies outside every
    # earlier sphere; every interior point lies inside some sphere
    assert np.all(np.diff(out.r) <= 0)
    for a in range(1, out.index.size):
        d2 = ((out.c[:a] - out.c[a]) ** 2).sum(1)
        assert np.all(d2 > out.r[:a] ** 2)
    d2 = ((pts[interior][:, None, :] - out.c[None]) ** 2).sum(-1)
    assert np.all((d2 <= out.r[None] ** 2).any(axis=1)) and out.n_left == 0
    # each centre is the deepest candidate (lowest index among equals) that
    # no earlier sphere covers
    cand = np.flatnonzero(interior)
    depth = np.abs(lv.S[cand])
    for a in range(out.index.size):
        free = np.ones(cand.size, bool)
        for q in range(a):
            free &= ((pts[cand] - out.c[q]) ** 2).sum(1) > out.r[q] ** 2
        top = depth[free].max()
        assert out.index[a] == cand[free][depth[free] == top].min()
    # eq. 3-11 holds at the nearest other centre's half distance
    d = np.exp(out.s[:, 0])
    assert np.allclose(out.w ** 2 * np.exp(-(d * out.dhat / 2) ** 2), 1e-3, rtol=1e-12)
    assert np.all(out.s[:, 0] == out.s[:, 1]) and np.all(out.s[:, 1] == out.s[:, 2])


def test_inscribed_sphere_init_cap_and_single_centre():
    lv = _sphere_level(16)
    full = O.inscribed_sphere_init([lv])
    part = O.inscribed_sphere_init([lv], m_max=3)
    assert np.array_equal(part.index, full.index[:3])
    pts = O.level_points(lv)
    interior = (lv.t > 1) & (lv.t < 2)
    d2 = ((pts[interior][:, None, :] - part.c[None]) ** 2).sum(-1)
    assert part.n_left == int((~(d2 <= part.r[None] ** 2).any(axis=1)).sum()) > 0
    one = O.inscribed_sphere_init([lv], m_max=1)
    assert one.dhat[0] == 2.0 and one.index.size == 1


def _plane_level(n, x0):
    ax = (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)
    z, y, x = np.meshgrid(ax.astype(np.float64), ax, ax, indexing="ij")
    return ax, (x - x0).astype(np.float32).reshape(-1)


def test_octree_mask_plane_count():
    # plane x = 0.1 on an 8^3 level: cell centres -0.875 ... 0.875 in steps of
    # 0.25; only x = 0.125 lies within sqrt(3)/8 = 0.2165 of the plane
    # (-0.125 is 0.225 away), so one slab of 64 parent cells is subdivided:
    # 512 children, in the two child x-slices 8 and 9 of 16
    _, S = _plane_level(8, 0.1)
    m = O.octree_mask(S, 8).reshape(16, 16, 16)
    assert m.sum() == 512
    assert np.all(m[:, :, 8:10]) and not m[:, :, :8].any() and not m[:, :, 10:].any()


def test_octree_mask_covers_the_surface_and_nests():
    # exact sphere distance: every cell of any depth that can meet the surface
    # (|S(centre)| <= its half-diagonal) is present, and a child is present
    # only under a present parent
    n0 = 6
    prev = None
    S_prev = _sphere_level(n0, 0.55).S
    for depth in range(3):
        n = n0 * 2 ** depth
        child = O.octree_mask(S_prev, n, prev)
        lv = _sphere_level(2 * n, 0.55)
        meets = np.abs(lv.S) <= np.sqrt(3.0) / (2 * n)
        if depth == 0:
            assert np.all(child[meets])
        else:
            # under the recursion a cell is present iff every ancestor may
            # meet the surface; cells meeting it have such ancestors
            assert np.all(child[meets])
            par = prev.reshape(n, n, n).repeat(2, 0).repeat(2, 1).repeat(2, 2).reshape(-1)
            assert not np.any(child & ~par)
        assert child.sum() < child.size
        prev, S_prev = child, lv.S


def test_targets_over_several_levels_keep_eq_3_10_on_its_branch():
    # eq. 3-10 uses the branch S >= m: with m the minimum over every level's
    # grid, each point of each level has S - m >= 0, the targets are a
    # non-increasing function of S over the union of the levels, and the
    # deepest point of any level gets t = 2.  A finer cell-centred grid comes
    # closer to a sphere's centre, so here the minimum lies on the second level.
    from synth.grid import axis_coords
    from synth.sdf import sample_sdf, sphere
    S = [sample_sdf([sphere(0.5)], axis_coords(n)).astype(np.float64) for n in (8, 16)]
    assert S[1].min() < S[0].min()
    m = O.sdf_min(S)
    allS = np.concatenate(S)
    assert np.all(allS - m >= 0.0)
    t = np.concatenate([O.targets_from_sdf(s, m) for s in S])
    order = np.argsort(allS, kind="stable")
    assert np.all(np.diff(t[order]) <= 1e-15)
    assert t.max() == pytest.approx(2.0, abs=1e-15)
