"""Pins for the oracle's loss, gradients, loss weights, Adam and seeding."""

import math

import numpy as np
import pytest

import oracle as O
import synth


def _problem(seed=0, n=12, m=5, lo=1.2, hi=2.0, wm=0, bands=None, orientation=0):
    p = synth.make_custom(seed, [n], m, (lo, hi), kinds=("ellipsoid", "torus"),
                          weight_map=wm, bands=bands, orientation=orientation)
    K = O.kernels_from_packed(p.params, p.m, p.cap, 3.0, wm, orientation)
    lv0 = p.levels[0]
    mS = O.sdf_min([lv0.S])
    t = O.targets_from_sdf(lv0.S, mS).astype(np.float32)
    lv = O.make_level(n, lv0.axis, active=lv0.active_mask(), t=t, S=lv0.S)
    return lv, K, p


# --- loss mask (eq. 3-18, eq. 3-19) ---------------------------------------

def test_loss_mask_hand_cases():
    # 8 points (n = 2); targets/predictions chosen so each rule fires once.
    t = np.array([1.0, 0.5, 0.5, 1.5, 1.5, 0.9, 1.1, 0.2])
    f = np.array([1.3, 0.95, 0.85, 1.05, 1.2, 0.91, 1.09, 0.2])
    lv = O.make_level(2, np.array([-0.5, 0.5]), t=t)
    K = O.make_kernels([0.5, -2.0], [[0, 0, 0]] * 2, [[0, 0, 0]] * 2, [[1, 0, 0, 0]] * 2, 3.0)
    lo = O.loss([lv], [f], K)
    # id0: 0.9<t<1.1 -> point 0; id1: t<=0.9 & f>0.9 -> points 1, 5;
    # id2: t>=1.1 & f<1.1 -> points 3, 6.
    expect = np.array([1, 1, 0, 1, 0, 1, 1, 0], bool)
    assert np.array_equal(lo.idall[0], expect)
    E = np.where(expect, f - t, 0.0)
    assert lo.L2 == pytest.approx(float(np.sum(E * E)), rel=1e-15)
    assert lo.max_abs_E == pytest.approx(0.45)
    assert lo.n_idall == 5
    assert lo.L1 == pytest.approx(2.5)


def test_loss_respects_active_mask():
    t = np.full(8, 1.0)
    f = np.linspace(0.5, 1.5, 8)
    act = np.array([1, 0, 1, 0, 1, 0, 1, 0], bool)
    lv = O.make_level(2, np.array([-0.5, 0.5]), active=act, t=t)
    K = O.make_kernels([1.0], [[0, 0, 0]], [[0, 0, 0]], [[1, 0, 0, 0]], 3.0)
    lo = O.loss([lv], [f], K)
    assert lo.n_idall == 4 and np.all(lo.E[0][~act] == 0)


# --- gradients -------------------------------------------------------------

def _fd_grads(lv, K, idall, h=1e-6, kernels=(0, 1, 2)):
    """Central differences of the all-pairs L2 with the mask frozen."""
    out = {}
    base = dict(w=K.w.copy(), c=K.c.copy(), s=K.s.copy(), q=K.q.copy())

    def L(fields):
        Kp = O.make_kernels(fields["w"], fields["c"], fields["s"], fields["q"], 3.0, K.weight_map, K.orientation)
        return O.l2_frozen([lv], Kp, idall, culled=False)

    for name, width in (("w", 1), ("c", 3), ("s", 3), ("q", 4)):
        g = np.zeros((len(kernels), width))
        for a, j in enumerate(kernels):
            for k in range(width):
                fp = {kk: vv.copy() for kk, vv in base.items()}
                fm = {kk: vv.copy() for kk, vv in base.items()}
                if name == "w":
                    fp["w"][j] += h
                    fm["w"][j] -= h
                else:
                    fp[name][j, k] += h
                    fm[name][j, k] -= h
                g[a, k] = (L(fp) - L(fm)) / (2 * h)
        out[name] = g
    return out


@pytest.mark.parametrize("wm,orientation", [(0, 0), (1, 0), (0, 1)])
def test_gradients_match_central_differences(wm, orientation):
    lv, K, _ = _problem(seed=11, n=12, m=5, wm=wm, orientation=orientation)
    assert np.all(np.abs(K.w) > 1e-4)
    f = O.forward([lv], K, culled=False)
    lo = O.loss([lv], f, K)
    assert lo.n_idall > 5
    G = [2.0 * e for e in lo.E]
    gr = O.backward([lv], K, G, culled=False)
    kern = (0, 2, 4)
    # the angle gradients are about 1e-4 of the loss, so the difference
    # quotient needs a wider step to stay above rounding (its truncation
    # error at 1e-4 is near 1e-8)
    fd = _fd_grads(lv, K, lo.idall, h=1e-4 if orientation else 1e-6, kernels=kern)
    ana = {"w": gr.w[list(kern)][:, None], "c": gr.c[list(kern)], "s": gr.s[list(kern)],
           "q": gr.q[list(kern)]}
    for name in ana:
        err = np.abs(ana[name] - fd[name]).max() / max(np.abs(fd[name]).max(), 1e-30)
        assert err < 1e-6, (name, err)


def _fd_combined(lv, K, idall, alpha, beta, h=1e-6, kernels=(0, 1, 2)):
    """Central differences of alpha * L2 + beta * L1 (eq. 3-14_2: L1 = sum |w|)
    with the mask and the weights (alpha, beta) frozen."""
    out = {}
    base = dict(w=K.w.copy(), c=K.c.copy(), s=K.s.copy(), q=K.q.copy())

    def J(fields):
        Kp = O.make_kernels(fields["w"], fields["c"], fields["s"], fields["q"], 3.0, K.weight_map, K.orientation)
        return alpha * O.l2_frozen([lv], Kp, idall, culled=False) + beta * float(np.sum(np.abs(fields["w"])))

    for name, width in (("w", 1), ("c", 3), ("s", 3), ("q", 4)):
        g = np.zeros((len(kernels), width))
        for a, j in enumerate(kernels):
            for k in range(width):
                fp = {kk: vv.copy() for kk, vv in base.items()}
                fm = {kk: vv.copy() for kk, vv in base.items()}
                if name == "w":
                    fp["w"][j] += h
                    fm["w"][j] -= h
                else:
                    fp[name][j, k] += h
                    fm[name][j, k] -= h
                g[a, k] = (J(fp) - J(fm)) / (2 * h)
        out[name] = g
    return out


@pytest.mark.parametrize("mode", ["fixed", "dynamic"])
def test_combined_gradient_matches_central_differences(mode):
    """eq. 3-15-2 / eq. 3-21: the step's gradient is alpha dL2 + beta dL1, the
    L1 term acting on w alone.  Pinned by central differences of
    alpha L2 + beta sum|w| itself, with |w| away from 0 so that |w| is
    differentiable; in the dynamic case alpha comes from eq. 3-21 and lies
    strictly inside (0, 1), so a dropped alpha or beta shows."""
    lv, K, _ = _problem(seed=15, n=12, m=5)
    assert np.all(np.abs(K.w) > 1e-4) and np.all(np.abs(np.abs(K.w) - 1.0) > 1e-3)
    f = O.forward([lv], K, culled=False)
    lo = O.loss([lv], f, K)
    G = [2.0 * e for e in lo.E]
    gr = O.backward([lv], K, G, culled=False)
    if mode == "fixed":
        al, be = O.loss_weights(O.MODE_FIXED, 0.37, False, lo.max_abs_E, 0.02, gr.w, K.w)
        assert (al, be) == (1.0, 0.37)
    else:
        # the gate of eq. l1_activate2 is opened with a tau_m above max|E|
        al, be = O.loss_weights(O.MODE_DYNAMIC, 0.0, True, lo.max_abs_E, lo.max_abs_E * 2 + 1.0, gr.w, K.w)
        assert 0.05 < al < 0.95 and be == pytest.approx(1.0 - al)
    comb = O.combine(gr, K.w, al, be)
    kern = (0, 2, 4)
    fd = _fd_combined(lv, K, lo.idall, al, be, kernels=kern)
    ana = {"w": comb.w[list(kern)][:, None], "c": comb.c[list(kern)], "s": comb.s[list(kern)],
           "q": comb.q[list(kern)]}
    # the quotient's rounding error is about 1e-16 |J| / h, up to 1e-6 of the
    # small orientation gradients here; a lost alpha or beta is an error of
    # at least 5 %
    for name in ana:
        err = np.abs(ana[name] - fd[name]).max() / max(np.abs(fd[name]).max(), 1e-30)
        assert err < 1e-5, (mode, name, err)


def test_culled_gradients_within_truncation_bounds():
    lv, K, _ = _problem(seed=12, n=16, m=8, lo=1.6, hi=2.4)
    f = O.forward([lv], K, culled=True)
    lo = O.loss([lv], f, K)
    G = [2.0 * e for e in lo.E]
    gc = O.backward([lv], K, G, culled=True)
    ga = O.backward([lv], K, G, culled=False)
    pts = O.level_points(lv)
    k2 = 9.0
    ek = math.exp(-k2)
    for j in range(K.m):
        out = np.sum((pts - K.c[j]) ** 2, axis=1) >= K.r2[j]
        sg = np.abs(G[0][out]).sum()
        a = abs(K.a[j])
        dmax, dmin = K.d[j].max(), K.d[j].min()
        assert abs(gc.a[j] - ga.a[j]) <= ek * sg * (1 + 1e-9) + 1e-300
        assert np.abs(gc.c[j] - ga.c[j]).max() <= 2 * a * dmax * 3.0 * ek * sg * (1 + 1e-9) + 1e-300
        assert np.abs(gc.s[j] - ga.s[j]).max() <= 2 * a * k2 * ek * sg * (1 + 1e-9) + 1e-300
        # dL/dR bound carried through the quaternion Jacobian
        J = O.quat_rot_jacobian(K.qhat[j:j + 1])[0].reshape(4, 9)
        rb = 2 * a * (dmax / dmin) * k2 * ek * sg
        assert np.linalg.norm(gc.q[j] - ga.q[j]) <= np.linalg.norm(J, 2) * rb / K.qn[j] * (1 + 1e-9) + 1e-300


def test_gradient_invariants():
    lv, K, _ = _problem(seed=13, n=12, m=6)
    rng = np.random.default_rng(3)
    G = [rng.standard_normal(lv.npts)]
    gr = O.backward([lv], K, G)
    # q . dL/dq = 0 (scale invariance of q)
    assert np.abs(np.sum(K.q * gr.q, axis=1)).max() < 1e-12 * max(1, np.abs(gr.q).max())
    # odd under q -> -q
    Kn = O.make_kernels(K.w, K.c, K.s, -K.q, 3.0)
    grn = O.backward([lv], Kn, G)
    assert np.abs(grn.q + gr.q).max() < 1e-12 * max(1, np.abs(gr.q).max())
    assert np.abs(grn.c - gr.c).max() < 1e-12 * max(1, np.abs(gr.c).max())
    # isotropic scales: orientation does not matter, so dL/dq = 0
    Ki = O.make_kernels(K.w, K.c, np.repeat(K.s[:, :1], 3, axis=1), K.q, 3.0)
    gi = O.backward([lv], Ki, G)
    assert np.abs(gi.q).max() < 1e-12
    # homogeneity: sum_j w_j dL/dw_j = 2 sum_i G_i f_i for a = w|w|
    f = O.forward([lv], K)
    assert np.sum(K.w * gr.w) == pytest.approx(2.0 * np.sum(G[0] * f[0]), rel=1e-12)
    KL = O.make_kernels(K.w, K.c, K.s, K.q, 3.0, weight_map=1)
    fL = O.forward([lv], KL)
    gL = O.backward([lv], KL, G)
    assert np.sum(KL.w * gL.w) == pytest.approx(np.sum(G[0] * fL[0]), rel=1e-12)


def test_single_isotropic_kernel_gradient_closed_form():
    lv = O.make_level(10, synth.axis_coords(10))
    pts = O.level_points(lv)
    c = np.array([0.05, -0.1, 0.15])
    dv, w = 2.5, -0.8
    K = O.make_kernels([w], [c], [[math.log(dv)] * 3], [[1, 0, 0, 0]], 3.0)
    G = np.random.default_rng(0).standard_normal(lv.npts)
    gr = O.backward([lv], K, [G], culled=False)
    delta = pts - c
    r2 = np.sum(delta ** 2, axis=1)
    phi = np.exp(-dv * dv * r2)
    a = w * abs(w)
    # f = a exp(-d^2 |x-c|^2): df/dc = 2 a d^2 (x - c) phi ; df/dw = 2|w| phi ;
    # with R = I each axis scale sees its own coordinate: df/ds_k = -2 a d^2 (x_k-c_k)^2 phi
    assert gr.w[0] == pytest.approx(np.sum(G * 2 * abs(w) * phi), rel=1e-12)
    assert np.allclose(gr.c[0], np.sum(G[:, None] * 2 * a * dv * dv * delta * phi[:, None], axis=0), rtol=1e-12)
    assert np.allclose(gr.s[0], np.sum(G[:, None] * -2 * a * dv * dv * delta ** 2 * phi[:, None], axis=0), rtol=1e-12)


# --- loss weights (eq. 3-21) ----------------------------------------------

def test_min_norm_alpha_closed_forms():
    e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    assert O.min_norm_alpha(g2=e2, g1=e1) == pytest.approx(0.5)
    assert O.min_norm_alpha(g2=np.zeros(3), g1=e1) == 1.0
    assert O.min_norm_alpha(g2=e2, g1=np.zeros(3)) == 0.0
    assert O.min_norm_alpha(g2=e1, g1=e1) == 1.0   # degenerate: documented reading


def test_min_norm_alpha_minimises_combined_norm():
    rng = np.random.default_rng(4)
    grid = np.linspace(0, 1, 20001)
    for _ in range(20):
        g2 = rng.standard_normal(30) * rng.uniform(0.01, 10)
        g1 = np.sign(rng.standard_normal(30))
        al = O.min_norm_alpha(g2, g1)
        norms = np.linalg.norm(grid[:, None] * g2[None] + (1 - grid[:, None]) * g1[None], axis=1)
        best = grid[np.argmin(norms)]
        assert abs(al - best) <= 1e-4


def test_loss_weights_gate():
    w = np.array([0.5, -0.2, 0.0])
    g = np.array([1.0, 2.0, 3.0])
    assert O.loss_weights(O.MODE_FIXED, 1e-4, False, 1.0, 0.02, g, w) == (1.0, 1e-4)
    assert O.loss_weights(O.MODE_DYNAMIC, 0, False, 0.0, 0.02, g, w) == (1.0, 0.0)
    assert O.loss_weights(O.MODE_DYNAMIC, 0, True, 0.03, 0.02, g, w) == (1.0, 0.0)
    al, be = O.loss_weights(O.MODE_DYNAMIC, 0, True, 0.01, 0.02, g, w)
    assert al == pytest.approx(O.min_norm_alpha(g, np.sign(w))) and be == pytest.approx(1 - al)
    assert np.array_equal(O.sign(np.array([-2.0, 0.0, 3.0])), [-1.0, 0.0, 1.0])


# --- Adam -------------------------------------------------------------------

def test_adam_matches_torch_fp64():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(7)]
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m1, m2 = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m1, m2 = O.adam_step(p, g, m1, m2, t, 1e-2)
    assert np.abs(p - tp.detach().numpy()).max() < 1e-14


# --- seeding (Algorithm 2, eq. 3-24) ---------------------------------------

def _seed_brute(levels, E, idall, top_frac, k_new, r_nms, eps):
    """Independent all-pairs restatement for tiny grids."""
    pts = np.concatenate([O.level_points(lv) for lv in levels])
    absE = np.abs(np.concatenate(E))
    ida = np.concatenate(idall)
    gid = np.flatnonzero(ida)
    K = math.ceil(top_frac * gid.size)
    ranked = sorted(gid, key=lambda g: (-absE[g], g))[:K]
    ranked = [g for g in ranked if absE[g] > eps]
    kept = []
    for g in ranked:
        d2 = np.sum((pts[gid] - pts[g]) ** 2, axis=1)
        if absE[g] >= absE[gid[d2 <= r_nms * r_nms]].max():
            kept.append(g)
    kept = sorted(kept, key=lambda g: (-absE[g], g))[:k_new]
    return np.array(kept, dtype=np.int64), pts


def test_seed_matches_brute_force_two_levels():
    rng = np.random.default_rng(6)
    lvs = []
    E, ida = [], []
    for n in (8, 16):
        ax = synth.axis_coords(n)
        S = rng.uniform(-0.2, 0.2, n ** 3)
        lvs.append(O.make_level(n, ax, S=S))
        e = np.round(rng.standard_normal(n ** 3), 2)  # rounding creates ties
        ia = rng.random(n ** 3) < 0.7
        E.append(np.where(ia, e, 0.0))
        ida.append(ia)
    out = O.seed(lvs, E, ida, top_frac=0.05, k_new=20, eps=1e-7)
    brute, pts = _seed_brute(lvs, E, ida, 0.05, 20, 2 * (2 / 16), 1e-7)
    assert np.array_equal(out.index, brute)
    # eq. 3-24 closed form: |E| exp(-d^2 dbar^2) = eps, centres at the points
    Eall = np.concatenate(E)
    Sall = np.concatenate([lv.S for lv in lvs])
    dbar = np.maximum(np.abs(Sall[brute]), 2 / 16)
    d = np.exp(out.s[:, 0])
    assert np.allclose(np.abs(Eall[brute]) * np.exp(-(d * dbar) ** 2), 1e-7, rtol=1e-10)
    assert np.array_equal(out.c, pts[brute])
    assert np.array_equal(out.w, -Eall[brute])
    assert np.all(out.q == [1, 0, 0, 0]) and np.all(out.s[:, 0] == out.s[:, 2])


def test_seed_single_peak_and_ties():
    n = 16
    ax = synth.axis_coords(n)
    lv = O.make_level(n, ax, S=np.zeros(n ** 3))
    pts = O.level_points(lv)
    # two equal peaks far apart, one smaller peak next to the first
    E = np.zeros(n ** 3)
    p1, p2 = 3 + 16 * (3 + 16 * 3), 12 + 16 * (12 + 16 * 12)
    E[p1] = 0.5
    E[p2] = -0.5
    E[p1 + 1] = 0.4
    ida = np.ones(n ** 3, bool)
    out = O.seed([lv], [E], [ida], top_frac=3 / n ** 3, k_new=10)
    # top-3 candidates: p1, p2 (tie -> lower index first), p1+1; the last is
    # suppressed by its neighbour p1
    assert list(out.index) == [p1, p2]
    assert np.array_equal(out.w, [-0.5, 0.5])
    assert out.n_candidates == 3 and out.n_extreme == 2
    assert np.array_equal(out.c[0], pts[p1])


def test_kernel_field_sums_to_forward_and_subset_gradients():
    lv, K, _ = _problem(seed=14, n=12, m=5)
    f = O.forward([lv], K)[0].reshape(lv.n, lv.n, lv.n)
    acc = np.zeros_like(f)
    for j in range(K.m):
        (z0, z1, y0, y1, x0, x1), v = O.kernel_field(lv, K, j)
        acc[z0:z1, y0:y1, x0:x1] += v
    assert np.abs(acc - f).max() < 1e-14
    G = [np.random.default_rng(1).standard_normal(lv.npts)]
    full = O.backward([lv], K, G)
    part = O.backward([lv], O.subset(K, [1, 3]), G)
    assert np.allclose(part.q, full.q[[1, 3]], rtol=1e-13, atol=0)
    assert np.allclose(part.c, full.c[[1, 3]], rtol=1e-13, atol=0)


def test_euler_isotropic_kernels_have_zero_angle_gradient():
    lv, K, p = _problem(seed=15, n=12, m=4, orientation=O.ORIENT_EULER)
    iso = O.make_kernels(K.w, K.c, np.repeat(K.s[:, :1], 3, axis=1), K.q, 3.0, 0, O.ORIENT_EULER)
    f = O.forward([lv], iso)
    lo = O.loss([lv], f, iso)
    gr = O.backward([lv], iso, [2.0 * e for e in lo.E])
    assert np.abs(gr.q).max() <= 1e-12 * max(1.0, np.abs(gr.c).max())
    assert np.all(gr.q[:, 3] == 0.0)


def test_batch_step_over_two_levels_is_additive():
    # batch indices run over the concatenation of the levels' points: a
    # partition of both levels' points into three batches adds up to the
    # full step, and a batch of the second level's points alone sees only them
    p = synth.make_custom(17, [8, 12], 6, (1.3, 2.1), kinds=("ellipsoid", "torus"))
    K = O.kernels_from_packed(p.params, p.m, p.cap, 3.0)
    mS = O.sdf_min([lv.S for lv in p.levels])
    levels = [O.make_level(lv.n, lv.axis, t=O.targets_from_sdf(lv.S, mS).astype(np.float32), S=lv.S)
              for lv in p.levels]
    n0, n1 = levels[0].npts, levels[1].npts
    full = O.step(levels, K)
    perm = np.random.default_rng(5).permutation(n0 + n1)
    parts = [O.step_batch(levels, K, perm[i::3]) for i in range(3)]
    assert abs(sum(b.loss.L2 for b in parts) - full.loss.L2) <= 1e-12 * full.loss.L2
    assert sum(b.loss.n_idall for b in parts) == full.loss.n_idall
    assert sum(b.P_fwd for b in parts) == full.P_fwd
    second = O.step_batch(levels, K, n0 + np.arange(n1))
    only = O.step([levels[1]], K)
    assert second.P_fwd == only.P_fwd and second.loss.n_idall == only.loss.n_idall


def test_batch_step_reduces_to_the_full_step_and_is_additive():
    lv, K, p = _problem(seed=16, n=12, m=6, lo=1.3, hi=2.1)
    full = O.step([lv], K)
    everything = O.step_batch([lv], K, np.arange(lv.npts))
    assert everything.loss.L2 == full.loss.L2 and everything.P_fwd == full.P_fwd
    assert np.array_equal(everything.grads.q, full.grads.q)
    # a partition into three batches: L2, counts and L2 gradients add up
    perm = np.random.default_rng(4).permutation(lv.npts)
    parts = [O.step_batch([lv], K, perm[i::3]) for i in range(3)]
    assert abs(sum(b.loss.L2 for b in parts) - full.loss.L2) <= 1e-12 * full.loss.L2
    assert sum(b.loss.n_idall for b in parts) == full.loss.n_idall
    assert sum(b.P_fwd for b in parts) == full.P_fwd and sum(b.P_bwd for b in parts) == full.P_bwd
    for k in ("w", "c", "s", "q"):
        tot = sum(getattr(b.grads_l2, k) for b in parts)
        ref = getattr(full.grads_l2, k)
        assert np.abs(tot - ref).max() <= 1e-12 * np.abs(ref).max()
    assert max(b.loss.max_abs_E for b in parts) == full.loss.max_abs_E


def test_culled_gradient_against_extended_radius_differences():
    """The culled analytic gradient of sum u f agrees with FP64 central
    differences taken on each kernel's field with the cull radius doubled,
    within the closed-form truncation allowance of the terms between r and
    2 r (the check the 512^3 GPU test applies to the device's gradient)."""
    from gpu_helpers import fd_check
    p = synth.make_custom(16, [24], 12, (1.6, 2.4), kinds=("ellipsoid", "torus"))
    lv0 = p.levels[0]
    lv = O.make_level(lv0.n, lv0.axis)
    K = O.kernels_from_packed(p.params, p.m, p.cap, p.cull_k)
    u = np.random.default_rng(4).standard_normal(lv.npts)
    gr = O.backward([lv], K, [u])
    grad = np.concatenate([gr.w[:, None], gr.c, gr.s, gr.q], axis=1)
    kk = np.repeat(np.arange(p.m), 11)
    pp = np.tile(np.arange(11), p.m)
    worst, exact, _ = fd_check(p, lv, u.reshape(lv.n, lv.n, lv.n), kk, pp, grad)
    for name in worst:
        assert worst[name] <= 1e-7 and exact[name] <= 1e-7, (name, worst[name], exact[name])
