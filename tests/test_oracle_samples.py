"""Pins for the oracle's surface samples P (label 1, the training set
V = {G, P} of Section 3.4.2): a sample set placed on grid points must give
exactly what the grid level gives there, by an independent code path (index
boxes against per-sample distances), and the sample-based inscribed-sphere
depth is the nearest-sample distance of a k-d tree."""

import numpy as np
from scipy.spatial import cKDTree

import oracle as O
import synth


def _grid_problem(seed=5, n=14, m=9):
    p = synth.make_custom(seed, [n], m, (1.4, 2.2), kinds=("ellipsoid", "torus"))
    K = O.kernels_from_packed(p.params, p.m, p.cap, 3.0, 0)
    lv0 = p.levels[0]
    mS = O.sdf_min([lv0.S])
    t = O.targets_from_sdf(lv0.S, mS).astype(np.float32)
    return O.make_level(n, lv0.axis, t=t, S=lv0.S), K


def _samples_on_grid(lv, seed, k=300, cap_extra=7):
    rng = np.random.default_rng(seed)
    pick = rng.choice(lv.npts, size=k, replace=False)
    return pick, O.make_samples(O.level_points(lv)[pick], cap=k + cap_extra)


def test_samples_on_grid_points_match_the_grid_forward_and_counts():
    lv, K = _grid_problem()
    pick, P = _samples_on_grid(lv, 1)
    f_grid = O.forward([lv], K)[0]
    f_s = O.forward([P], K)[0]
    assert f_s.shape == (P.cap,) and np.all(f_s[len(pick):] == 0.0)
    assert np.allclose(f_s[:len(pick)], f_grid[pick], rtol=1e-13, atol=1e-15)
    # in-ball pair counts: restrict the grid level to the picked points
    act = np.zeros(lv.npts, bool)
    act[pick] = True
    sub = O.make_level(lv.n, lv.axis, active=act, t=lv.t, S=lv.S)
    G_grid = np.zeros(lv.npts)
    G_grid[pick] = np.linspace(-1.0, 1.0, len(pick))
    G_s = np.zeros(P.cap)
    G_s[:len(pick)] = G_grid[pick]
    assert O.pair_counts([sub], K, [G_grid]) == O.pair_counts([P], K, [G_s])
    # truncation bound and boundary allowance at the same points
    tb_g, tb_s = O.truncation_bound([lv], K)[0], O.truncation_bound([P], K)[0]
    assert np.allclose(tb_s[:len(pick)], tb_g[pick], rtol=1e-13, atol=1e-300)
    al_g, _ = O.boundary_allowance([sub], K)
    al_s, _ = O.boundary_allowance([P], K)
    assert np.allclose(al_s[0][:len(pick)], al_g[0][pick], rtol=1e-13, atol=1e-300)


def test_samples_on_grid_points_match_the_grid_gradients():
    lv, K = _grid_problem(seed=6)
    pick, P = _samples_on_grid(lv, 2)
    rng = np.random.default_rng(3)
    G_grid = np.zeros(lv.npts)
    G_grid[pick] = rng.normal(size=len(pick))
    G_s = np.zeros(P.cap)
    G_s[:len(pick)] = G_grid[pick]
    g_grid = O.backward([lv], K, [G_grid])
    g_s = O.backward([P], K, [G_s])
    for name in ("w", "c", "s", "q", "a"):
        a, b = getattr(g_s, name), getattr(g_grid, name)
        assert np.allclose(a, b, rtol=1e-11, atol=1e-12 * np.abs(b).max()), name


def test_sample_loss_uses_label_one():
    lv, K = _grid_problem(seed=7)
    pick, P = _samples_on_grid(lv, 4)
    f = O.forward([P], K)
    lo = O.loss([P], f, K, 0.9, 1.1)
    k = len(pick)
    # tau1 < 1 < tau2: every sample is in id_all with E = f - 1
    assert lo.n_idall == k and np.all(lo.idall[0][:k]) and not lo.idall[0][k:].any()
    assert lo.L2 == np.sum((f[0][:k] - 1.0) ** 2)


def test_step_batch_partition_with_samples():
    # the batches of a partition of grid points and samples add up to the
    # full step (L2 and the L2 gradient)
    lv, K = _grid_problem(seed=8, n=10)
    pick, P = _samples_on_grid(lv, 5, k=120)
    levels = [lv, P]
    full = O.step(levels, K, mode=O.MODE_L2)
    pts = np.concatenate([np.arange(lv.npts), lv.npts + np.arange(len(pick))])
    parts = np.array_split(np.random.default_rng(9).permutation(pts), 3)
    L2 = 0.0
    gw = np.zeros(K.m)
    for b in parts:
        st = O.step_batch(levels, K, b, mode=O.MODE_L2)
        L2 += st.loss.L2
        gw += st.grads.w
    assert np.isclose(L2, full.loss.L2, rtol=1e-12)
    assert np.allclose(gw, full.grads.w, rtol=1e-10, atol=1e-12 * np.abs(full.grads.w).max())


def test_init_depth_from_samples_is_the_nearest_sample_distance():
    # exact sphere distance; samples on the sphere: the depth of each
    # interior point is its squared distance to the nearest sample (k-d tree)
    n = 16
    ax = (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)
    z, y, x = np.meshgrid(ax.astype(np.float64), ax, ax, indexing="ij")
    S = (np.sqrt(x * x + y * y + z * z) - 0.6).astype(np.float32).reshape(-1)
    t = O.targets_from_sdf(S, O.sdf_min([S])).astype(np.float32)
    lv = O.make_level(n, ax, t=t, S=S)
    rng = np.random.default_rng(11)
    v = rng.normal(size=(400, 3))
    sp = (0.6 * v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    P = O.make_samples(sp, cap=410)
    out = O.inscribed_sphere_init([lv, P])
    interior = np.flatnonzero((lv.t > 1) & (lv.t < 2))
    d, _ = cKDTree(P.pts).query(O.level_points(lv)[interior])
    depth = dict(zip(interior.tolist(), (d * d).tolist()))
    # every centre is the deepest uncovered candidate by that depth (float32
    # order, lowest index among equals), and the radii are those depths
    pts = O.level_points(lv)
    key = {i: np.float32(depth[i]) for i in interior}
    for a, k in enumerate(out.index):
        assert np.isclose(out.r[a] ** 2, depth[int(k)], rtol=1e-12)
        free = [i for i in interior
                if all(((pts[i] - out.c[q]) ** 2).sum() > out.r[q] ** 2 * (1 + 1e-12) for q in range(a))]
        top = max(key[i] for i in free)
        assert k == min(i for i in free if key[i] == top)
    assert out.n_left == 0 and out.index.size > 5


def _sphere_level_and_samples(n=16, k=400, cap=410, seed=11):
    ax = (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)
    z, y, x = np.meshgrid(ax.astype(np.float64), ax, ax, indexing="ij")
    S = (np.sqrt(x * x + y * y + z * z) - 0.6).astype(np.float32).reshape(-1)
    lv = O.make_level(n, ax, S=S)
    v = np.random.default_rng(seed).normal(size=(k, 3))
    sp = (0.6 * v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    return lv, O.make_samples(sp, cap=cap)


def test_seed_with_samples_matches_all_pairs_and_eq_3_24():
    """Algorithm 2 on V = {G, P}: the neighbourhoods hold the id_all samples
    as well as the grid points, samples are not candidates, and eq. 3-24's
    dbar is the distance to the nearest sample (a k-d tree here), floored at
    the grid spacing.  Restated by all pairs over V."""
    lv, P = _sphere_level_and_samples()
    rng = np.random.default_rng(12)
    Eg = np.round(rng.normal(size=lv.npts), 2) * (np.abs(lv.S) < 0.3)
    Es = np.zeros(P.cap)
    Es[:P.pts.shape[0]] = np.round(rng.normal(size=P.pts.shape[0]), 2)
    ida_g, ida_s = Eg != 0.0, P.act() & (Es != 0.0)
    r_nms = 0.3
    out = O.seed([lv, P], [Eg, Es], [ida_g, ida_s], top_frac=0.05, k_new=30, r_nms=r_nms, eps=1e-7)
    # all pairs over V
    X = np.concatenate([O.level_points(lv), O.level_points(P)])
    absE = np.abs(np.concatenate([Eg, Es]))
    ida = np.concatenate([ida_g, ida_s])
    grid = np.arange(X.shape[0]) < lv.npts
    K = int(np.ceil(0.05 * ida.sum()))
    ranked = sorted(np.flatnonzero(ida & grid), key=lambda g: (-absE[g], g))[:K]
    kept = []
    for g in ranked:
        if absE[g] <= 1e-7:
            continue
        nb = np.flatnonzero(ida & (np.nansum((X - X[g]) ** 2, axis=1) <= r_nms * r_nms))
        if absE[g] >= absE[nb].max():
            kept.append(g)
    kept = sorted(kept, key=lambda g: (-absE[g], g))[:30]
    assert list(out.index) == kept and len(kept) >= 5
    # the samples did suppress: without them more grid candidates survive
    alone = O.seed([lv], [Eg], [ida_g], top_frac=0.05, k_new=30, r_nms=r_nms, eps=1e-7,
                   n_idall=int(ida.sum()))
    assert alone.n_extreme > out.n_extreme
    # eq. 3-24: |E| exp(-d^2 dbar^2) = eps with dbar the nearest-sample distance
    dist, _ = cKDTree(P.pts).query(out.c)
    dbar = np.maximum(dist, 2.0 / lv.n)
    d = np.exp(out.s[:, 0])
    assert np.allclose(absE[out.index] * np.exp(-(d * dbar) ** 2), 1e-7, rtol=1e-10)
    assert np.array_equal(out.w, -np.concatenate([Eg, Es])[out.index])


def test_seed_samples_suppress_but_are_not_chosen():
    lv, P = _sphere_level_and_samples(k=50, cap=50)
    pts = O.level_points(lv)
    Eg = np.zeros(lv.npts)
    Es = np.zeros(P.cap)
    # grid peak next to a sample with a larger |E| (suppressed), a second grid
    # peak with no sample near it (kept), and the largest |E| of all on a
    # sample (never a candidate)
    s0 = P.pts[0]
    g_near = int(np.argmin(np.sum((pts - s0) ** 2, axis=1)))
    far = np.sum((P.pts[:, None, :] - pts[None, :, :]) ** 2, axis=2).min(axis=0)
    g_far = int(np.argmax(np.where(np.abs(lv.S) < 0.2, far, -1.0)))
    Eg[g_near], Eg[g_far] = 0.5, -0.4
    Es[0], Es[1] = 0.7, 0.9
    r = float(np.sqrt(np.sum((pts[g_near] - s0) ** 2))) * 1.01
    assert r < np.sqrt(far[g_far])
    ida_g, ida_s = Eg != 0, Es != 0
    out = O.seed([lv, P], [Eg, Es], [ida_g, ida_s], top_frac=1.0, k_new=10, r_nms=r)
    assert list(out.index) == [g_far]
    assert out.n_candidates == 2 and out.n_extreme == 1
