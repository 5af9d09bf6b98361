"""GPU-vs-oracle parity at full problem sizes.

* the 256^3 timing snapshot (16384 ERBFs on 64^3 + 128^3 + band(256^3)) in
  the launch configuration the benchmark times, element by element over all
  19M points and all kernels (the oracle runs over kernel chunks in worker
  processes);
* the 128^3 / 2048-ERBF problem with eq. 3-21 active, element by element;
* every tile of a 128^3 and a 256^3 level (36 864 slots, packed sort keys
  with the sign bit set), element by element;
* the 512^3 / 65536-ERBF problem through the autograd path, on sampled
  points (f) and sampled kernels (gradients for a seeded upstream).

Bars as in the small cases: f within 1e-5 of ||f||_inf plus each point's
cull-boundary allowance, gradients per group within 1e-4, counts exact
(pair counts up to the boundary-ambiguous pairs, which are reported).
"""

import time

import numpy as np
import pytest

import oracle as O
from oracle import pool as oracle_pool
import synth
from gpu_helpers import TAU1, TAU2, TAU_M, GpuProblem, fd_check, oracle_grads_dict, oracle_levels, record, rel_inf

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

F_TOL = 1e-5
G_TOL = 1e-4


def _torch():
    import torch
    return torch


def _say(*a):
    print(*a, flush=True)


def _full_step_case(name, prob, pair_cap, mode, l1_active, tau_m, lam=0.0):
    torch = _torch()
    t0 = time.perf_counter()
    olv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32, pair_cap=pair_cap)
    G = torch.zeros(gp.ctx.n_points, dtype=torch.float32, device=gp.ctx.device)
    f = torch.zeros_like(G)
    _say(f"{name}: loss_grad on the GPU, {gp.ctx.n_points} points, {prob.m} kernels")
    g = gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, mode=mode, lam=lam, l1_active=l1_active, tau1=TAU1, tau2=TAU2,
                              tau_m=tau_m, f_out=f, G_out=G)
    torch.cuda.synchronize()
    st = gp.ctx.stats()[0]
    fl, Gl, gg = gp.split_points(f), gp.split_points(G), gp.grads_np(g)
    del gp, f, G, g
    torch.cuda.empty_cache()
    _say(f"{name}: GPU done; oracle over {oracle_pool.workers()} workers")
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ref = oracle_pool.step(olv, K, mode=mode, lam=lam, l1_active=l1_active, tau1=TAU1, tau2=TAU2, tau_m=tau_m)
    _say(f"{name}: oracle done ({time.perf_counter() - t0:.1f} s since set-up)")

    fmax = max(np.abs(x).max() for x in ref.f)
    e_f = max(float(((np.abs(a.astype(np.float64) - b) - al) / fmax).max()) for a, b, al in zip(fl, ref.f, ref.allow))
    # mask decisions that float32 and float64 could take differently
    amb_pts = 0
    for lv, fo in zip(olv, ref.f):
        near = ((np.abs(fo - TAU1) < 1e-5) & (lv.t <= TAU1)) | ((np.abs(fo - TAU2) < 1e-5) & (lv.t >= TAU2))
        amb_pts += int((near & lv.act()).sum())
    # G = 2E at every point (0 off the mask)
    e_G = 0.0
    for a, b, al in zip(Gl, ref.G, ref.allow):
        e_G = max(e_G, float(((np.abs(a.astype(np.float64) - b) - 2 * al) / (2 * fmax)).max()))
        assert np.array_equal(a != 0, b != 0)
    errs = dict(
        e_f=e_f, e_G=e_G,
        L2=abs(st.L2 - ref.loss.L2) / ref.loss.L2,
        L1=abs(st.L1 - ref.loss.L1) / ref.loss.L1,
        max_abs_E=abs(st.max_abs_E - ref.loss.max_abs_E),
        alpha=abs(st.alpha - ref.alpha), beta=abs(st.beta - ref.beta))
    go = oracle_grads_dict(ref.grads)
    for k in go:
        errs["grad_" + k] = rel_inf(gg[k], go[k])
    record(name, n_idall=(st.n_idall, ref.loss.n_idall), P_fwd=(st.P_fwd, ref.P_fwd), P_bwd=(st.P_bwd, ref.P_bwd),
           boundary_pairs=ref.n_amb, mask_ambiguous_points=amb_pts, alpha_value=ref.alpha, **errs)
    assert amb_pts == 0, "workload has float-ambiguous mask decisions"
    assert st.flags == 0
    assert st.n_idall == ref.loss.n_idall
    assert abs(st.P_fwd - ref.P_fwd) <= ref.n_amb and abs(st.P_bwd - ref.P_bwd) <= ref.n_amb
    assert e_f <= F_TOL and e_G <= F_TOL
    assert errs["L2"] <= 1e-5 and errs["L1"] <= 1e-5 and errs["max_abs_E"] <= 1e-5
    assert errs["alpha"] <= 1e-5 and errs["beta"] <= 1e-5
    for k in go:
        assert errs["grad_" + k] <= G_TOL, (k, errs["grad_" + k])
    return st, ref


def test_large_snapshot_full_parity_in_bench_configuration():
    from paper_2505_02350_amd.fit import ShapeInput, estimate_pair_cap
    prob = synth.make_large_snapshot()
    s = ShapeInput.from_problem(prob)
    cap = estimate_pair_cap(s.level_ns, s.s_min(), prob.cull_k)   # as the benchmark's Fitter sizes it
    _full_step_case("full_large_snapshot", prob, cap, O.MODE_DYNAMIC, True, TAU_M)


def test_mid_full_parity_min_norm_weights():
    prob = synth.make_mid()
    st, ref = _full_step_case("full_mid_dynamic", prob, None, O.MODE_DYNAMIC, True, 10.0)
    assert 0.0 < ref.alpha <= 1.0


def test_packed_sort_keys_with_slots_from_2_15():
    """Every tile of a 128^3 and a 256^3 level: 4096 + 32768 = 36864 tile
    slots and 512 kernels, so the sort keys carry slot << 16 | kernel in one
    32-bit word, and the slots of the 256^3 level's top eighth in z (32768
    and up) set its sign bit.  Element-by-element parity with the oracle, as
    above, with balls reaching those tiles."""
    prob = synth.make_custom(108, [128, 256], 512, (3.4, 3.8))
    slots = sum((lv.n // 8) ** 3 for lv in prob.levels)
    assert slots == 36864 and prob.cap <= 65536
    P = np.asarray(prob.params, np.float64).reshape(11, prob.cap)[:, :prob.m]
    r = prob.cull_k / np.exp(P[4:7].min(axis=0))
    # slot 4096 + t is at least 32768 from the 256^3 tile row tz = 28 on
    z_top = prob.levels[1].axis[28 * 8]
    reach = int((P[3] + r > z_top).sum())
    _say(f"{reach} kernels reach the tiles of slot 32768 and up")
    assert reach >= 8
    _full_step_case("full_packed_keys_high_slots", prob, None, O.MODE_FIXED, False, TAU_M, lam=1e-4)


def test_diff_512_autograd_sampled_parity():
    """512^3, 65536 ERBFs: f on sampled points; gradients of sampled kernels
    for a seeded upstream gradient (the oracle evaluates those kernels only)."""
    torch = _torch()
    from paper_2505_02350_amd.autograd import ERBFLayer
    t0 = time.perf_counter()
    prob = synth.make_diff()
    _say(f"diff workload generated in {time.perf_counter() - t0:.1f} s")
    lv = prob.levels[0]
    n = lv.n
    gp = GpuProblem(prob, None)
    layer = ERBFLayer(gp.ctx, gp.p, gp.m_dev)
    rng = np.random.default_rng(2024)
    u = rng.standard_normal(n ** 3, dtype=np.float32)
    ut = torch.from_numpy(u).to(gp.ctx.device)
    _say("diff: autograd forward + backward on the GPU")
    f = layer()
    (f * ut).sum().backward()
    torch.cuda.synchronize()
    del ut
    fg = f.detach().cpu().numpy()
    gg = gp.grads_np(layer.p.grad)
    del f, layer, gp
    torch.cuda.empty_cache()

    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ax = np.asarray(lv.axis, np.float64)
    # points: half uniform over the grid, half near sampled kernel centres
    n_pts = 2000
    idx_u = rng.choice(n ** 3, n_pts // 2, replace=False)
    jc = rng.choice(prob.m, n_pts // 2, replace=True)
    near = np.clip(np.rint((K.c[jc] + 1.0) * n / 2.0 - 0.5).astype(np.int64)
                   + rng.integers(-4, 5, size=(n_pts // 2, 3)), 0, n - 1)
    idx_n = near[:, 0] + n * (near[:, 1] + n * near[:, 2])
    idx = np.concatenate([idx_u, idx_n])
    pts = np.stack([ax[idx % n], ax[(idx // n) % n], ax[idx // (n * n)]], axis=1)
    _say(f"diff: oracle f at {len(idx)} points")
    f_or = O.forward_at_points(pts, K)
    allow, n_amb = O.allowance_at_points(pts, K)
    fmax = np.abs(f_or).max()
    e_f = float(((np.abs(fg[idx].astype(np.float64) - f_or) - allow) / fmax).max())

    js = np.sort(rng.choice(prob.m, 512, replace=False))
    _say(f"diff: oracle gradients of {len(js)} kernels")
    olv = O.make_level(n, lv.axis)
    gr = O.backward([olv], O.subset(K, js), [u.astype(np.float64)])
    go = oracle_grads_dict(gr)
    errs = {k: rel_inf(gg[k][js], go[k]) for k in go}
    record("diff_512_autograd_sampled", e_f=e_f, f_inf_sampled=fmax, boundary_pairs=n_amb, n_points=len(idx),
           n_kernels=len(js), **errs)
    assert e_f <= F_TOL
    for k in go:
        assert errs[k] <= G_TOL, (k, errs[k])

    # FP64 central differences of sum_i u_i f_i for 1000 random (kernel,
    # parameter) pairs (250 kernels, 4 parameters each), each on the kernel's own field with the cull radius
    # doubled, against the GPU gradient within the truncation allowance of
    # the terms between r and 2 r (see gpu_helpers.fd_check)
    _say("diff: finite differences of 1000 parameters")
    u3 = u.reshape(n, n, n)
    kk = np.repeat(rng.choice(prob.m, 250, replace=False), 4)
    pp = np.concatenate([rng.choice(11, 4, replace=False) for _ in range(250)])
    gpu_all = np.concatenate([gg["w"][:, None], gg["c"], gg["s"], gg["q"]], axis=1)
    worst, exact, max_allow = fd_check(prob, olv, u3, kk, pp, gpu_all)
    record("diff_512_finite_differences", n_params=int(kk.size), worst_minus_allowance=worst,
           worst_with_exact_shell=exact, max_allowance_rel=max_allow)
    for name, e in exact.items():
        assert e <= G_TOL, (name, e)
    for name, e in worst.items():
        assert e <= G_TOL, (name, e)


def test_seed_at_large_snapshot_size():
    """Algorithm 2 at the 256^3 snapshot's size (64^3 + 128^3 + band(256^3),
    5.8 M training points, a third of them in id_all with a seeded residual):
    top 1 % candidates (about 19 000), extreme points, the first 256 kernels,
    against the oracle."""
    torch = _torch()
    prob = synth.make_large_snapshot()
    prob.cap = prob.m + 256
    prob.params = np.concatenate([prob.params.reshape(11, prob.m), np.zeros((11, 256), np.float32)],
                                 axis=1).reshape(-1)
    olv, t32, _ = oracle_levels(prob)
    rng = np.random.default_rng(37)
    E, ida = [], []
    for lv in olv:
        e = (np.round(rng.standard_normal(lv.npts) * 0.3, 2)).astype(np.float32)
        ia = lv.act() & (rng.random(lv.npts) < 0.33)
        E.append(np.where(ia, e, np.float32(0)).astype(np.float32))
        ida.append(ia & (E[-1] != 0))
    n_id = int(sum(i.sum() for i in ida))
    tf = float(np.float32(0.01))
    _say(f"seed at full size: {n_id} id_all points, oracle")
    out = O.seed(olv, [e.astype(np.float64) for e in E], ida, top_frac=tf, k_new=256)
    gp = GpuProblem(prob, t32, pair_cap=1 << 20)
    resid = torch.from_numpy(np.concatenate(E)).to(gp.ctx.device)
    _say("seed at full size: GPU")
    n = gp.ctx.erbf_seed_from_error(gp.p, gp.m_dev, 0, resid, 1.0, n_id, top_frac=tf, k_new=256)
    torch.cuda.synchronize()
    P = gp.p.cpu().numpy().reshape(11, prob.cap)
    new = P[:, prob.m:prob.m + n]
    s_err = float(np.abs(new[4:7].T.astype(np.float64) - out.s).max() / max(1.0, np.abs(out.s).max()))
    record("seed_large_snapshot", n_idall=n_id, n_candidates=out.n_candidates, n_added=n, s_rel_err=s_err)
    assert n == out.index.size == 256
    assert np.array_equal(new[0], out.w.astype(np.float32))
    assert np.array_equal(new[1:4].T, out.c.astype(np.float32))
    assert np.array_equal(new[7:11].T, out.q.astype(np.float32))
    assert s_err <= 1e-6
