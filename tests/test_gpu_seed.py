"""GPU parity of seeding (Algorithm 2, eq. 3-24) and of refining (eq. 3-16)."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import TAU1, TAU2, GpuProblem, oracle_levels, record, rel_inf

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _residual_field(lvs, seed, frac=0.7, decimals=2):
    rng = np.random.default_rng(seed)
    E, ida = [], []
    for lv in lvs:
        e = np.round(rng.standard_normal(lv.npts) * 0.3, decimals).astype(np.float32)
        ia = rng.random(lv.npts) < frac
        E.append(np.where(ia, e, np.float32(0.0)).astype(np.float32))
        ida.append(ia)
    return E, ida


def _seed_case(name, levels_n, k_new, top_frac, seed, m0=16, cap=600, min_abs_err=0.0, w_rule=0, bands=None,
               orientation=0):
    torch = _torch()
    prob = synth.make_custom(seed, levels_n, m0, (1.5, 2.5), bands=bands, cap=cap, orientation=orientation)
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    E, ida = _residual_field(olv, seed + 100)
    tf = float(np.float32(top_frac))
    out = O.seed(olv, [e.astype(np.float64) for e in E], ida, top_frac=tf, k_new=k_new,
                 min_abs_err=float(np.float32(min_abs_err)), w_rule=w_rule, orientation=orientation)
    resid = torch.from_numpy(np.concatenate(E)).to(gp.ctx.device)
    m1 = torch.full((11 * gp.ctx.cap_total,), 7.0, device=gp.ctx.device)
    m2 = torch.full_like(m1, 9.0)
    n_id = int(sum(i.sum() for i in ida))
    n = gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, resid, 1.0, n_id, top_frac=tf, k_new=k_new,
                                    min_abs_err=min_abs_err, w_rule=w_rule, m1=m1, m2=m2)
    torch.cuda.synchronize()
    assert n == out.index.size, (n, out.index.size)
    assert int(gp.m_dev.item()) == m0 + n
    p = gp.p.cpu().numpy().reshape(11, cap)
    new = p[:, m0:m0 + n]
    assert np.array_equal(new[0], out.w.astype(np.float32))
    assert np.array_equal(new[1:4].T, out.c.astype(np.float32))
    assert np.array_equal(new[7:11].T, out.q.astype(np.float32))
    s_err = float(np.abs(new[4:7].T.astype(np.float64) - out.s).max() / max(1.0, np.abs(out.s).max())) if n else 0.0
    assert s_err <= 1e-6
    # untouched kernels and cleared moments
    assert np.array_equal(p[:, :m0], prob.params.reshape(11, cap)[:, :m0])
    mm1 = m1.cpu().numpy().reshape(11, cap)
    assert np.all(mm1[:, m0:m0 + n] == 0.0) and np.all(mm1[:, :m0] == 7.0) and np.all(mm1[:, m0 + n:] == 7.0)
    record(name, n_added=n, n_candidates=out.n_candidates, n_extreme=out.n_extreme, s_rel_err=s_err)
    return gp, out


def test_seed_two_levels_matches_oracle():
    _seed_case("seed_two_levels", [16, 32], k_new=64, top_frac=0.02, seed=31)


def test_seed_k_new_limits_and_sqrt_rule():
    _seed_case("seed_knew", [24], k_new=5, top_frac=0.05, seed=32, w_rule=1)


def test_seed_euler_orientation_writes_zero_angles():
    gp, out = _seed_case("seed_euler", [16, 24], k_new=32, top_frac=0.02, seed=36, orientation=1)
    assert out.index.size > 0 and not np.any(out.q)


def test_seed_min_abs_err_floor():
    _seed_case("seed_floor", [16, 24], k_new=256, top_frac=0.05, seed=33, min_abs_err=0.7)


def test_seed_capacity_error_leaves_state():
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    prob = synth.make_custom(34, [16], 16, (1.5, 2.5), cap=20)
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    E, ida = _residual_field(olv, 134)
    resid = torch.from_numpy(np.concatenate(E)).to(gp.ctx.device)
    p0 = gp.p.clone()
    with pytest.raises(L.ErbfError) as ei:
        gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, resid, 1.0, int(sum(i.sum() for i in ida)),
                                    top_frac=0.05, k_new=64)
    assert ei.value.code == L.ERBF_ERR_CAPACITY
    torch.cuda.synchronize()
    assert int(gp.m_dev.item()) == 16 and torch.equal(gp.p, p0)


def test_seed_after_loss_uses_G():
    """Seeding from the loss pass's own G (E = G / 2) equals the oracle on the
    oracle's E of the same step."""
    torch = _torch()
    prob = synth.make_custom(35, [16, 32], 24, (1.6, 2.6), bands=[None, 0.2], cap=400)
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    G = torch.zeros(gp.ctx.n_points, device=gp.ctx.device)
    gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, tau1=TAU1, tau2=TAU2, G_out=G)
    torch.cuda.synchronize()
    st = gp.ctx.stats()[0]
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    f = O.forward(olv, K)
    lo = O.loss(olv, f, K, TAU1, TAU2)
    assert st.n_idall == lo.n_idall
    # the kernel ranks |E| in float32: the oracle ranks its own residuals
    # rounded to float32 the same way
    E32 = [e.astype(np.float32).astype(np.float64) for e in lo.E]
    out = O.seed(olv, E32, lo.idall, top_frac=float(np.float32(0.01)), k_new=32)
    # smallest gap between consecutive |E| in the ranked top part: recorded,
    # since a near-tie there could let float32 rounding flip a decision
    absE = np.sort(np.abs(np.concatenate(E32))[np.concatenate(lo.idall)])[::-1]
    gaps = np.abs(np.diff(absE[:int(np.ceil(0.01 * lo.n_idall)) + 1]))
    n = gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, G, 0.5, st.n_idall, top_frac=0.01, k_new=32)
    torch.cuda.synchronize()
    Eg = [0.5 * g for g in gp.split_points(G)]
    for eg, eo in zip(Eg, lo.E):
        assert np.abs(eg - eo).max() <= 1e-5 * max(1.0, np.abs(eo).max())
    record("seed_after_loss", n_added=n, n_oracle=int(out.index.size), min_gap=float(gaps.min()) if gaps.size else None)
    assert n == out.index.size
    p = gp.p.cpu().numpy().reshape(11, prob.cap)
    assert np.array_equal(p[1:4, 24:24 + n].T, out.c.astype(np.float32))
    assert np.allclose(p[0, 24:24 + n], out.w, rtol=1e-5, atol=1e-6)


def test_refine_appends_levels():
    """Training set grows level by level (eq. 3-16): after each append the
    step equals the oracle's on the union of the levels registered so far."""
    torch = _torch()
    from paper_2505_02350_amd import core
    prob = synth.make_custom(36, [8, 16, 32], 20, (1.6, 2.6), bands=[None, None, 0.2])
    olv, t32, _ = oracle_levels(prob)
    dev = torch.device("cuda")
    ctx = core.Context([([lv.n for lv in prob.levels], prob.cap)], 1 << 16, prob.cull_k)
    p = torch.from_numpy(prob.params).to(dev)
    mdev = torch.tensor([prob.m], dtype=torch.int32, device=dev)
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    keep = []
    for li, lv in enumerate(prob.levels):
        S = torch.from_numpy(lv.S).to(dev)
        bits = core.erbf_band_bits(S, lv.band) if lv.band is not None else None
        ax = torch.from_numpy(lv.axis).to(dev)
        t = torch.from_numpy(t32[li]).to(dev)
        keep.append((S, bits, ax, t))
        ctx.erbf_refine_level(0, ax, t, S, bits)
        g = ctx.erbf_loss_grad(p, mdev, lam=1e-3, tau1=TAU1, tau2=TAU2)
        torch.cuda.synchronize()
        st = ctx.stats()[0]
        ref = O.step(olv[:li + 1], K, mode=O.MODE_FIXED, lam=1e-3, tau1=TAU1, tau2=TAU2)
        assert st.n_idall == ref.loss.n_idall and st.P_fwd == ref.P_fwd and st.P_bwd == ref.P_bwd
        assert abs(st.L2 - ref.loss.L2) <= 1e-5 * ref.loss.L2
        gg = g.cpu().numpy().astype(np.float64).reshape(11, prob.cap)[:, :prob.m]
        go = ref.grads.packed(prob.cap).reshape(11, prob.cap)[:, :prob.m]
        # per parameter group, each against its own scale (a small group such
        # as q must not hide behind a large one)
        for name, sl in (("w", slice(0, 1)), ("c", slice(1, 4)), ("s", slice(4, 7)), ("q", slice(7, 11))):
            assert rel_inf(gg[sl], go[sl]) <= 1e-4, (li, name, rel_inf(gg[sl], go[sl]))
    # registering past the declared levels is an error
    from paper_2505_02350_amd import _lib as L
    with pytest.raises((L.ErbfError, IndexError)):
        ctx.erbf_refine_level(0, keep[0][2])
