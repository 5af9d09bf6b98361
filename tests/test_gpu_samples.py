"""Surface samples P (label 1; the training set V = {G, P} of Section 3.4.2)
on the device against the oracle: the full step with a sample level between
two grid levels, one crowded sample tile, the VJP, a mini-batch mixing grid
points and samples, seeding with samples in the neighbourhoods and dbar, and the inscribed-sphere
initialisation with the nearest-sample depth of Algorithm 1."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import TAU1, TAU2, GpuProblem, oracle_grads_dict, oracle_levels, record, rel_inf
from test_gpu_parity import _loss_case

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _problem(seed, nbin=32, count=3000, cap=3010, levels=(16, 24), m=40, kcap=None):
    return synth.make_custom(seed, list(levels), m, (1.6, 2.6), kinds=("ellipsoid", "torus", "capsule"),
                             samples=(1, count, nbin, cap), cap=kcap)


def test_step_with_samples_between_grid_levels():
    prob = _problem(81)
    gp, g, st = _loss_case("loss_samples", prob, O.MODE_DYNAMIC, l1_active=True, tau_m=10.0)
    # every sample is a training point with label 1
    assert st.n_idall >= 3000


def test_step_with_one_crowded_sample_tile():
    # an 8-cell binning grid: all 5000 samples share one tile (several
    # 256-sample passes in the forward, several 1024-sample stages in the
    # backward)
    prob = _problem(82, nbin=8, count=5000, cap=5000)
    _loss_case("loss_samples_one_tile", prob, O.MODE_FIXED, lam=1e-4)


def test_vjp_with_samples():
    torch = _torch()
    prob = _problem(83)
    olv, t32, _ = oracle_levels(prob, with_targets=False)
    gp = GpuProblem(prob, None)
    rng = np.random.default_rng(4)
    up = rng.normal(size=gp.ctx.n_points).astype(np.float32)
    g = gp.ctx.erbf_vjp(gp.p, gp.m_dev, torch.from_numpy(up).to(gp.ctx.device))
    torch.cuda.synchronize()
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    G, base = [], 0
    for lv in olv:
        G.append(np.where(lv.act(), up[base:base + lv.npts].astype(np.float64), 0.0))
        base += lv.npts
    ref = O.backward(olv, K, G)
    go, gg = oracle_grads_dict(ref), gp.grads_np(g)
    errs = {k: rel_inf(gg[k], go[k]) for k in go}
    record("vjp_samples", **errs)
    for k in go:
        assert errs[k] <= 1e-4, (k, errs[k])


def test_minibatch_mixing_grid_points_and_samples():
    torch = _torch()
    prob = _problem(84)
    olv, t32, _ = oracle_levels(prob)
    pts, base = [], 0
    for lv in olv:
        pts.append(base + np.nonzero(lv.act())[0])
        base += lv.npts
    pts = np.concatenate(pts).astype(np.int64)
    batch = np.random.default_rng(6).permutation(pts)[: int(0.3 * pts.size)]
    gp = GpuProblem(prob, t32, batch_cap=batch.size)
    f = torch.zeros(batch.size, device=gp.ctx.device)
    kw = dict(mode=O.MODE_FIXED, lam=1e-4, tau1=TAU1, tau2=TAU2)
    g = gp.ctx.erbf_loss_grad_minibatch(gp.p, gp.m_dev, torch.from_numpy(batch).to(gp.ctx.device), f_out=f, **kw)
    torch.cuda.synchronize()
    st = gp.ctx.stats()[0]
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ref = O.step_batch(olv, K, batch, **kw)
    f_or = np.concatenate(ref.f)[batch]
    e_f = float(np.abs(f.cpu().numpy() - f_or).max() / np.abs(f_or).max())
    go, gg = oracle_grads_dict(ref.grads), gp.grads_np(g)
    errs = {k: rel_inf(gg[k], go[k]) for k in go}
    n_samp = int(((batch >= gp.ctx.pt_base[0][1]) & (batch < gp.ctx.pt_base[0][2])).sum())
    record("minibatch_samples", e_f=e_f, batch_samples=n_samp, n_idall=(st.n_idall, ref.loss.n_idall),
           P_fwd=(st.P_fwd, ref.P_fwd), P_bwd=(st.P_bwd, ref.P_bwd), **errs)
    assert n_samp > 100
    assert e_f <= 1e-5
    assert st.n_idall == ref.loss.n_idall and st.P_fwd == ref.P_fwd and st.P_bwd == ref.P_bwd
    assert abs(st.L2 - ref.loss.L2) <= 1e-5 * ref.loss.L2
    for k in go:
        assert errs[k] <= 1e-4, (k, errs[k])


def test_seeding_with_samples_matches_oracle():
    # Algorithm 2 on V = {G, P}: registered samples sit in the extreme-point
    # neighbourhoods and give eq. 3-24's dbar (nearest-sample distance);
    # they are never candidates
    torch = _torch()
    prob = _problem(85, kcap=400)
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    rng = np.random.default_rng(7)
    E, ida = [], []
    for lv in olv:
        if isinstance(lv, O.OSamples):
            e = np.zeros(lv.npts, np.float32)
            e[:lv.pts.shape[0]] = np.round(rng.normal(size=lv.pts.shape[0]) * 0.6, 2)
        else:
            e = np.round(rng.normal(size=lv.npts) * 0.3, 2).astype(np.float32)
            e[rng.random(lv.npts) < 0.3] = 0.0
        E.append(e.astype(np.float32))
        ida.append(e != 0.0)
    n_id = int(sum(i.sum() for i in ida))
    tf = float(np.float32(0.02))
    out = O.seed(olv, [e.astype(np.float64) for e in E], ida, top_frac=tf, k_new=1024, eps=1e-7,
                 n_idall=n_id)
    grid_only = O.seed([lv for lv in olv if not isinstance(lv, O.OSamples)],
                       [e.astype(np.float64) for e, lv in zip(E, olv) if not isinstance(lv, O.OSamples)],
                       [i for i, lv in zip(ida, olv) if not isinstance(lv, O.OSamples)], top_frac=tf, k_new=1024,
                       eps=1e-7, n_idall=n_id)
    # the samples change the result: fewer extreme points, other scales
    assert out.n_extreme < grid_only.n_extreme
    resid = torch.from_numpy(np.concatenate(E)).to(gp.ctx.device)
    n = gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, resid, 1.0, n_id, top_frac=tf, k_new=1024, eps=1e-7)
    torch.cuda.synchronize()
    assert n == out.index.size > 10
    P = gp.p.cpu().numpy().reshape(11, prob.cap)
    new = P[:, prob.m:prob.m + n]
    assert np.array_equal(new[0], out.w.astype(np.float32))
    assert np.array_equal(new[1:4].T, out.c.astype(np.float32))
    assert np.array_equal(new[7:11].T, out.q.astype(np.float32))
    s_err = float(np.abs(new[4:7].T.astype(np.float64) - out.s).max() / max(1.0, np.abs(out.s).max()))
    record("seed_with_samples", n_added=n, n_candidates=out.n_candidates, n_extreme=out.n_extreme,
           n_extreme_grid_only=grid_only.n_extreme, s_rel_err=s_err)
    assert s_err <= 1e-6


def test_init_with_samples_uses_the_nearest_sample_depth():
    torch = _torch()
    prob = _problem(86, nbin=32, count=2000, cap=2000)
    prob.cap = 4096
    prob.params = np.zeros(11 * prob.cap, np.float32)
    prob.m = 0
    lv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32, pair_cap=1 << 20)
    nc, left = gp.ctx.erbf_init_inscribed(gp.p, gp.m_dev, 0, gamma=float(np.float32(1e-3)))
    torch.cuda.synchronize()
    ref = O.inscribed_sphere_init(lv, gamma=float(np.float32(1e-3)), m_max=prob.cap)
    assert nc == ref.index.size > 10 and left == ref.n_left
    P = gp.p.cpu().numpy().reshape(11, prob.cap)[:, :nc].astype(np.float64)
    assert np.array_equal(P[0], ref.w) and np.array_equal(P[1:4].T, ref.c)
    err_s = float(np.abs(P[4:7].T - ref.s).max())
    record("init_samples", centres=nc, left=left, err_s=err_s)
    assert err_s <= 1e-6 * max(1.0, float(np.abs(ref.s).max()))


def test_sample_level_edges():
    torch = _torch()
    from paper_2505_02350_amd import core, _lib as L
    prob = synth.make_custom(87, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus"))
    olv, t32, _ = oracle_levels(prob)
    dev = torch.device("cuda")

    def ctx_with(samples):
        ctx = core.Context([([16, 8, 24], prob.cap, [0, 64, 0])], 1 << 22, prob.cull_k)
        for li, lv in ((0, prob.levels[0]), (1, None), (2, prob.levels[1])):
            if lv is None:
                ctx.erbf_refine_samples(0, torch.from_numpy(samples).to(dev))
            else:
                ctx.erbf_refine_level(0, torch.from_numpy(lv.axis).to(dev), torch.from_numpy(t32[0 if li == 0 else 1]).to(dev),
                                      torch.from_numpy(lv.S).to(dev))
        return ctx

    p = torch.from_numpy(prob.params).to(dev)
    m = torch.tensor([prob.m], dtype=torch.int32, device=dev)
    # no samples registered: the grid results equal a context without the level
    ctx0 = ctx_with(np.zeros((0, 3), np.float32))
    g0 = ctx0.erbf_loss_grad(p, m, mode=O.MODE_FIXED, lam=1e-4)
    plain = core.Context([([16, 24], prob.cap)], 1 << 22, prob.cull_k)
    for li in range(2):
        lv = prob.levels[li]
        plain.erbf_refine_level(0, torch.from_numpy(lv.axis).to(dev), torch.from_numpy(t32[li]).to(dev),
                                torch.from_numpy(lv.S).to(dev))
    g1 = plain.erbf_loss_grad(p, m, mode=O.MODE_FIXED, lam=1e-4)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)
    # samples on the corners and faces of the domain
    corners = np.array([[1, 1, 1], [-1, -1, -1], [1, -1, 0.5], [0, 0, 1], [-1, 0.25, 0]], np.float32)
    ctx1 = ctx_with(corners)
    f = torch.zeros(ctx1.n_points, device=dev)
    ctx1.erbf_loss_grad(p, m, mode=O.MODE_FIXED, lam=1e-4, f_out=f)
    torch.cuda.synchronize()
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ref = O.forward([O.make_samples(corners, 64)], K)[0]
    base = ctx1.pt_base[0][1]
    got = f[base:base + 64].cpu().numpy()
    allow, _ = O.boundary_allowance([O.make_samples(corners, 64)], K)
    assert np.all(np.abs(got - ref) <= 1e-5 * max(1.0, np.abs(ref).max()) + allow[0])
    # invalid samples are rejected before anything is registered
    bad = core.Context([([16, 8], prob.cap, [0, 4])], 1 << 20, prob.cull_k)
    bad.erbf_refine_level(0, torch.from_numpy(prob.levels[0].axis).to(dev), torch.from_numpy(t32[0]).to(dev),
                          torch.from_numpy(prob.levels[0].S).to(dev))
    with pytest.raises(L.ErbfError):
        bad.erbf_refine_samples(0, torch.tensor([[0.0, 1.5, 0.0]], device=dev))
    with pytest.raises(L.ErbfError):
        bad.erbf_refine_samples(0, torch.zeros((5, 3), device=dev))
