"""Edge cases of the HIP path, each checked against the oracle: no kernels,
an empty training mask (id_all of eq. 3-18 empty), bucket-list overflow,
kernels whose ball misses the domain, isotropic kernels (rotation gradient
zero) and unnormalised quaternions."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import (TAU1, TAU2, GpuProblem, oracle_grads_dict, oracle_levels, pair_cap_estimate, record,
                         rel_inf)
from test_gpu_parity import _loss_case

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _no_kernels(cull_k):
    z = np.zeros((0, 3))
    return O.make_kernels(np.zeros(0), z, z, np.zeros((0, 4)), cull_k)


def test_no_kernels_then_seed_the_first_ones():
    """M = 0: f = 0 everywhere, E = -t on id_all, zero gradients; seeding
    from that residual then places the first kernels (Algorithm 2)."""
    torch = _torch()
    prob = synth.make_custom(51, [12, 20], 8, (1.6, 2.6), bands=[None, 0.2], cap=64)
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    m0 = torch.zeros(1, dtype=torch.int32, device=gp.ctx.device)
    f = gp.ctx.erbf_eval(gp.p, m0)
    G = torch.full((gp.ctx.n_points,), 5.0, device=gp.ctx.device)
    f2 = torch.full_like(G, 5.0)
    g = gp.ctx.erbf_loss_grad(gp.p, m0, mode=O.MODE_FIXED, lam=1e-4, tau1=TAU1, tau2=TAU2, f_out=f2, G_out=G)
    torch.cuda.synchronize()
    st = gp.ctx.stats()[0]
    ref = O.step(olv, _no_kernels(prob.cull_k), mode=O.MODE_FIXED, lam=1e-4, tau1=TAU1, tau2=TAU2)
    assert not f.any() and not f2.any() and not g.any()
    assert st.P_fwd == 0 and st.P_bwd == 0 and st.flags == 0
    assert st.n_idall == ref.loss.n_idall > 0
    assert abs(st.L2 - ref.loss.L2) <= 1e-6 * ref.loss.L2 and st.L1 == 0.0
    # E = 0 - t is exact in float32, so G = 2E is too
    for gl, gr in zip(gp.split_points(G), ref.G):
        assert np.array_equal(gl.astype(np.float64), gr)
    E32 = [e.astype(np.float32).astype(np.float64) for e in ref.loss.E]
    out = O.seed(olv, E32, ref.loss.idall, top_frac=float(np.float32(0.02)), k_new=40)
    n = gp.ctx.erbf_seed_from_error(gp.p, m0, 0, G, 0.5, st.n_idall, top_frac=0.02, k_new=40)
    torch.cuda.synchronize()
    record("edge_no_kernels", n_idall=st.n_idall, L2=(st.L2, ref.loss.L2), n_seeded=(n, int(out.index.size)))
    assert n == out.index.size > 0 and int(m0.item()) == n
    p = gp.p.cpu().numpy().reshape(11, prob.cap)
    assert np.array_equal(p[1:4, :n].T, out.c.astype(np.float32))
    assert np.array_equal(p[0, :n], out.w.astype(np.float32))


def test_empty_training_mask():
    """Targets all below tau1 and f below tau1 everywhere: id_all is empty,
    L2 = 0 and only the L1 part of eq. 3-21 moves the weights."""
    torch = _torch()
    prob = synth.make_custom(52, [16], 12, (1.6, 2.6))
    olv, _, _ = oracle_levels(prob)
    t_low = [np.full(lv.npts, 0.5, np.float32) for lv in olv]
    olv = [O.make_level(lv.n, lv.axis, active=lv.active, t=t, S=lv.S) for lv, t in zip(olv, t_low)]
    gp = GpuProblem(prob, t_low)
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    for mode, lam in ((O.MODE_FIXED, 1e-3), (O.MODE_DYNAMIC, 0.0)):
        g = gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, mode=mode, lam=lam, l1_active=True, tau1=TAU1, tau2=TAU2,
                                  tau_m=0.02)
        torch.cuda.synchronize()
        st = gp.ctx.stats()[0]
        ref = O.step(olv, K, mode=mode, lam=lam, l1_active=True, tau1=TAU1, tau2=TAU2, tau_m=0.02)
        assert ref.loss.n_idall == 0 and max(np.abs(x).max() for x in ref.f) < TAU1
        assert st.n_idall == 0 and st.L2 == 0.0 and st.max_abs_E == 0.0 and st.P_bwd == 0
        assert st.P_fwd == ref.P_fwd
        assert abs(st.alpha - ref.alpha) <= 1e-6 and abs(st.beta - ref.beta) <= 1e-6
        gg, go = gp.grads_np(g), oracle_grads_dict(ref.grads)
        assert rel_inf(gg["w"], go["w"]) <= 1e-6
        for k in ("c", "s", "q"):
            assert not np.any(gg[k])
    n = gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, torch.zeros(gp.ctx.n_points, device=gp.ctx.device), 1.0,
                                    0, top_frac=0.01, k_new=8)
    assert n == 0 and int(gp.m_dev.item()) == prob.m


def test_bucket_overflow_is_flagged_and_counted():
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    prob = synth.make_custom(53, [16, 24], 20, (1.5, 2.5))
    _, t32, _ = oracle_levels(prob)
    small = GpuProblem(prob, t32, pair_cap=64)
    small.ctx.erbf_loss_grad(small.p, small.m_dev, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    st_s = small.ctx.stats()[0]
    big = GpuProblem(prob, t32)
    big.ctx.erbf_loss_grad(big.p, big.m_dev, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    st_b = big.ctx.stats()[0]
    record("edge_overflow", needed=st_s.n_bucket_pairs, cap=64)
    assert st_s.flags & L.FLAG_BUCKET_OVERFLOW
    assert st_b.flags == 0
    assert st_s.n_bucket_pairs == st_b.n_bucket_pairs > 64


def _edit_params(prob, fn):
    p = prob.params.reshape(11, prob.cap).copy()
    fn(p)
    prob.params = p.reshape(-1).astype(np.float32)
    return prob


def test_outside_domain_and_isotropic_kernels():
    def edit(p):
        p[1:4, 0] = (1.9, 0.0, 0.0)        # ball misses the domain
        p[1:4, 1] = (-1.02, 0.3, -0.2)     # centre just outside, ball reaches in
        p[4:7, 2] = 2.0                    # isotropic: rotation cannot change f
        p[4:7, 3] = 1.7
    prob = _edit_params(synth.make_custom(54, [16, 24], 16, (1.5, 2.5), bands=[None, 0.25]), edit)
    gp, g, st = _loss_case("edge_outside_isotropic", prob, O.MODE_FIXED, lam=1e-4)
    gg = gp.grads_np(g)
    # the ball misses every grid point: only the L1 term reaches its weight
    assert not np.any(gg["c"][0]) and not np.any(gg["s"][0]) and not np.any(gg["q"][0])
    assert gg["w"][0] == np.float32(1e-4) * np.sign(prob.params[0])
    scale = np.abs(gg["c"]).max()
    assert np.abs(gg["q"][2:4]).max() <= 1e-6 * scale


def test_unnormalised_quaternions():
    """q and 3q describe the same rotation: f agrees and dL/dq scales by 1/3
    (the gradient is taken through q / |q|)."""
    torch = _torch()
    prob = synth.make_custom(55, [20], 16, (1.5, 2.5))

    def triple_q(p):
        p[7:11] *= 3.0
    prob3 = _edit_params(synth.make_custom(55, [20], 16, (1.5, 2.5)), triple_q)
    outs = []
    for pr in (prob, prob3):
        _, t32, _ = oracle_levels(pr)
        gp = GpuProblem(pr, t32)
        f = torch.zeros(gp.ctx.n_points, device=gp.ctx.device)
        g = gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, lam=1e-4, tau1=TAU1, tau2=TAU2, f_out=f)
        torch.cuda.synchronize()
        outs.append((f.cpu().numpy(), gp.grads_np(g)))
    (f1, g1), (f3, g3) = outs
    assert np.abs(f1 - f3).max() <= 1e-6 * np.abs(f1).max()
    assert rel_inf(3.0 * g3["q"], g1["q"]) <= 1e-4
    for k in ("w", "c", "s"):
        assert rel_inf(g3[k], g1[k]) <= 1e-4
    olv, _, _ = oracle_levels(prob3)
    K3 = O.kernels_from_packed(prob3.params, prob3.m, prob3.cap, prob3.cull_k)
    ref = O.step(olv, K3, mode=O.MODE_FIXED, lam=1e-4, tau1=TAU1, tau2=TAU2)
    assert rel_inf(g3["q"], ref.grads.q) <= 1e-4


def test_bucket_total_past_2_31_is_flagged_and_counted():
    """The bucket-entry offsets are 64-bit: 70 000 kernels whose balls
    (radius 6) reach all 32^3 tiles of a 256^3 grid need 70 000 * 32 768 =
    2 293 760 000 entries, more than 2^31.  The count comes back exactly,
    the overflow flag is raised, and nothing past the small list capacity is
    written."""
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd import core
    n, m = 256, 70000
    ctx = core.Context([([n], m)], pair_cap=1 << 20, cull_k=3.0)
    dev = ctx.device
    ax = torch.from_numpy(synth.axis_coords(n)).to(dev)
    ctx.erbf_refine_level(0, ax)
    rng = np.random.default_rng(56)
    p = np.zeros((11, m), np.float32)
    p[0] = rng.uniform(0.1, 0.2, m)
    p[1:4] = rng.uniform(-1.0, 1.0, (3, m))
    p[4:7] = np.float32(np.log(0.5))
    p[7] = 1.0
    pt = torch.from_numpy(p.reshape(-1)).to(dev)
    mdev = torch.tensor([m], dtype=torch.int32, device=dev)
    print("256^3 grid, 70000 kernels of radius 6, pair_cap 2^20", flush=True)
    ctx.erbf_eval(pt, mdev, stats=True)
    torch.cuda.synchronize()
    st = ctx.stats()[0]
    record("edge_offsets_64bit", needed=st.n_bucket_pairs, cap=1 << 20)
    assert st.n_bucket_pairs == m * (n // 8) ** 3 > 2 ** 31
    assert st.flags & L.FLAG_BUCKET_OVERFLOW
    ctx.close()


def _host_tile_counts(prob):
    """Tiles of 8^3 points whose point box each kernel's cull ball reaches
    (float64, no widening), over every level; all tiles active."""
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k, prob.weight_map, prob.orientation)
    r2 = K.r2
    out = np.zeros(len(r2), int)
    for lv in prob.levels:
        ax = np.asarray(lv.axis, np.float64)
        t = np.arange((lv.n + 7) // 8)
        lo, hi = ax[8 * t], ax[np.minimum(8 * t + 7, lv.n - 1)]
        for j in range(len(r2)):
            e = [np.maximum(np.maximum(lo - K.c[j, d], K.c[j, d] - hi), 0.0) for d in range(3)]
            d2 = e[2][:, None, None] ** 2 + e[1][None, :, None] ** 2 + e[0][None, None, :] ** 2
            out[j] += int((d2 < r2[j]).sum())
    return out


def test_kept_tile_slots_and_walked_kernels_agree():
    """The count pass keeps at most hit_cap = min(512, 2 pair_cap / capacity)
    tile slots per kernel and the emit pass copies them; a kernel with more
    tiles is walked again.  With the list capacity exactly the step's entry
    count, kernels of both kinds occur (scales spread over e^1.2 .. e^4); the
    gradient and the statistics equal bit for bit those of a context where
    every kernel copies, which the oracle checks."""
    torch = _torch()
    prob = synth.make_custom(67, [40], 64, (1.2, 4.0), cap=64)
    _, g_all, st_all = _loss_case("edge_hit_cap", prob, O.MODE_FIXED, lam=1e-4)
    E = st_all.n_bucket_pairs
    hit_cap = min(512, 2 * E // prob.cap)
    counts = _host_tile_counts(prob)
    record("edge_hit_cap_mix", entries=E, hit_cap=hit_cap, walked=int((counts > hit_cap).sum()),
           max_tiles=int(counts.max()))
    assert 16 <= hit_cap < 512
    assert (counts > hit_cap + 2).sum() >= 3 and (counts < hit_cap - 2).sum() >= 3
    # the oracle-checked context (default capacity) keeps every kernel's slots
    assert min(512, 2 * pair_cap_estimate(prob) // prob.cap) > counts.max() + 2
    _, t32, _ = oracle_levels(prob)
    tight = GpuProblem(prob, t32, pair_cap=E)
    g = tight.ctx.erbf_loss_grad(tight.p, tight.m_dev, mode=O.MODE_FIXED, lam=1e-4, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    st = tight.ctx.stats()[0]
    assert st.flags == 0 and st.n_bucket_pairs == E
    assert (st.L2, st.L1, st.P_fwd, st.P_bwd, st.n_idall) == (st_all.L2, st_all.L1, st_all.P_fwd, st_all.P_bwd,
                                                               st_all.n_idall)
    assert torch.equal(g, g_all)
