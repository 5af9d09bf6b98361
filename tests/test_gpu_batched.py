"""The batching extension: many shapes in one context (one launch per stage),
launch variants, the autotuner and HIP-graph replay."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import TAU1, TAU2, oracle_grads_dict, oracle_levels, record, rel_inf

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _shapes(n=4, seed=50):
    out = []
    for b in range(n):
        ns = [[16], [24], [12, 20], [32]][b % 4]
        bands = [None] * (len(ns) - 1) + ([0.2] if b % 2 else [None])
        out.append(synth.make_custom(seed + b, ns, 12 + 7 * b, (1.6, 2.6), kinds=("ellipsoid", "torus"),
                                     bands=bands, cap=16 + 8 * b))
    return out


def _fitter(probs):
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    return Fitter([ShapeInput.from_problem(p) for p in probs], cull_k=3.0)


def _shape_grad(fit, g, b):
    cap_total = fit.ctx.cap_total
    kb = fit.ctx.kbase[b]
    cap = fit.shapes[b].cap
    return g.detach().cpu().numpy().reshape(11, cap_total)[:, kb:kb + cap]


def test_batched_equals_plain_bitwise_and_variants():
    torch = _torch()
    probs = _shapes()
    lams = torch.tensor([1e-5, 1e-4, 1e-3, 1e-4], device="cuda")
    fb = _fitter(probs)
    outs = {}
    keys = [(v, c, r, 256, 4, o) for v in range(8) for c in (0, 8) for r in (1, 0) for o in (1, 0)]
    keys += [(v, 8, 0, ch, w, 1) for v in (0, 3) for ch in (64, 128, 256) for w in (2, 4, 8)]
    for v, c, r, ch, w, o in keys:
        print(f"batched loss_grad, 4 shapes, launch variant {v}, XCD runs {c}, ranked lists {r}, "
              f"forward chunk {ch}, backward waves {w}, longest tiles first {o}", flush=True)
        fb.ctx.erbf_set_launch(v, c, 16, r, ch, w, o)
        g = fb.ctx.erbf_loss_grad_batched(fb.p, fb.m_dev, lambda_dev=lams, tau1=TAU1, tau2=TAU2)
        torch.cuda.synchronize()
        outs[(v, c, r, ch, w, o)] = (g.clone(), fb.ctx.stats())
    for k in keys[1:]:
        assert torch.equal(outs[k][0], outs[keys[0]][0]), k
        assert all(a.P_bwd == b.P_bwd and a.P_fwd == b.P_fwd and a.L2 == b.L2
                   for a, b in zip(outs[k][1], outs[keys[0]][1])), k
    fb.ctx.erbf_set_launch(0, 8, 16, 1)
    gb, stb = outs[keys[0]]
    for b, p in enumerate(probs):
        fp = _fitter([p])
        gpl = fp.ctx.erbf_loss_grad(fp.p, fp.m_dev, lam=float(lams[b]), tau1=TAU1, tau2=TAU2)
        torch.cuda.synchronize()
        stp = fp.ctx.stats()[0]
        assert np.array_equal(_shape_grad(fb, gb, b), _shape_grad(fp, gpl, 0)), b
        assert stb[b].L2 == stp.L2 and stb[b].P_fwd == stp.P_fwd and stb[b].P_bwd == stp.P_bwd
        assert stb[b].n_idall == stp.n_idall and stb[b].beta == stp.beta


def test_batched_matches_oracle():
    torch = _torch()
    probs = _shapes(3, seed=60)
    lams = [1e-5, 1e-4, 1e-3]
    fb = _fitter(probs)
    g = fb.ctx.erbf_loss_grad(fb.p, fb.m_dev, lambda_dev=torch.tensor(lams, device="cuda"), tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    st = fb.ctx.stats()
    for b, p in enumerate(probs):
        olv, _, _ = oracle_levels(p)
        K = O.kernels_from_packed(p.params, p.m, p.cap, p.cull_k)
        ref = O.step(olv, K, mode=O.MODE_FIXED, lam=lams[b], tau1=TAU1, tau2=TAU2)
        a = _shape_grad(fb, g, b).astype(np.float64)[:, :p.m]
        gg = {"w": a[0], "c": a[1:4].T, "s": a[4:7].T, "q": a[7:11].T}
        go = oracle_grads_dict(ref.grads)
        errs = {k: rel_inf(gg[k], go[k]) for k in go}
        record(f"batched_shape{b}", **errs)
        assert st[b].n_idall == ref.loss.n_idall and st[b].P_fwd == ref.P_fwd
        for k in go:
            assert errs[k] <= 1e-4, (b, k, errs[k])


def test_graph_replay_matches_eager():
    torch = _torch()
    probs = _shapes(3, seed=70)
    kw = dict(lam=1e-4, lr=1e-3, tau1=TAU1, tau2=TAU2)
    fe = _fitter(probs)
    fg = _fitter(probs)
    fg.capture(**kw)          # runs one eager warm-up step, then captures one step
    fe.step(**kw)             # keep both fitters at the same step count
    for it in range(4):
        fe.step(**kw)
        fg.replay()
        # eager work on the default stream between replays
        torch.cuda.synchronize()
        _ = (fe.p * 2).sum().item()
        assert torch.equal(fe.p, fg.p), it
        assert torch.equal(fe.m1, fg.m1) and torch.equal(fe.step_dev, fg.step_dev)


def test_autotune_picks_a_variant_and_keeps_results():
    torch = _torch()
    probs = _shapes(4, seed=80)
    fb = _fitter(probs)
    g0 = fb.ctx.erbf_loss_grad(fb.p, fb.m_dev, lam=1e-4, tau1=TAU1, tau2=TAU2).clone()
    p0 = fb.p.clone()
    v, times = fb.ctx.erbf_autotune(fb.p, fb.m_dev, reps=2, lam=1e-4, tau1=TAU1, tau2=TAU2)
    timed = [t for t in times if t >= 0]
    assert 0 <= v < 8 and fb.ctx.erbf_get_variant() == v and times[v] >= 0
    assert len(timed) == 6 and all(t > 0 for t in timed)
    launch = fb.ctx.erbf_get_launch()
    print("autotuned launch:", launch, flush=True)
    assert launch["variant"] == v and launch["fwd_chunk"] in (64, 128, 256) and launch["bwd_waves"] in (2, 4, 8)
    assert launch["tile_order"] in (0, 1)
    assert torch.equal(fb.p, p0)
    g1 = fb.ctx.erbf_loss_grad(fb.p, fb.m_dev, lam=1e-4, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)


@pytest.mark.parametrize("mode", ["fixed", "dynamic"])
def test_train_step_equals_loss_grad_then_adam(mode):
    """erbf_train_step (eq. 3-21 combination applied inside the Adam pass)
    gives bit for bit the parameters, moments, step counters and combined
    gradient of erbf_loss_grad followed by erbf_adam_step, step after step."""
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    probs = _shapes(4, seed=90)
    fa, fb = _fitter(probs), _fitter(probs)
    lams = torch.tensor([1e-5, 1e-4, 1e-3, 1e-4], device="cuda")
    kw = dict(mode=L.MODE_FIXED, lambda_dev=lams) if mode == "fixed" else \
        dict(mode=L.MODE_DYNAMIC, l1_active=True, tau_m=10.0)
    lr = torch.tensor([1e-2, 5e-3, 1e-2, 2e-3], device="cuda")
    for it in range(4):
        print(f"train step {it} ({mode})", flush=True)
        fa.ctx.erbf_train_step(fa.p, fa.m_dev, fa.grad, fa.m1, fa.m2, fa.step_dev, lr_dev=lr, tau1=TAU1, tau2=TAU2,
                               **kw)
        fb.ctx.erbf_loss_grad(fb.p, fb.m_dev, grad_out=fb.grad, tau1=TAU1, tau2=TAU2, **kw)
        fb.ctx.erbf_adam_step(fb.p, fb.m_dev, fb.grad, fb.m1, fb.m2, fb.step_dev, lr_dev=lr)
        torch.cuda.synchronize()
        for name in ("p", "grad", "m1", "m2", "step_dev"):
            assert torch.equal(getattr(fa, name), getattr(fb, name)), (it, name)
        sa, sb = fa.stats(), fb.stats()
        for b in range(4):
            assert sa[b].L2 == sb[b].L2 and sa[b].alpha == sb[b].alpha and sa[b].beta == sb[b].beta
    assert fa.step_dev.cpu().tolist() == [4, 4, 4, 4]
    if mode == "dynamic":
        assert any(0.0 < s.alpha < 1.0 for s in fa.stats())


@pytest.mark.timeout(900)
def test_batching_config_extreme_shapes_match_oracle():
    """The 64-shape batching workload (grids 32^3..128^3, 256..4096 kernels,
    per-shape lambda) in one batched context; the shapes with the most and
    the fewest points x kernels against the oracle (f-derived counts exact,
    gradients per group within 1e-4)."""
    torch = _torch()
    from oracle import pool
    print("batching workload: generating 64 shapes", flush=True)
    probs = synth.make_batching()
    fb = _fitter(probs)
    lams = torch.tensor([p.lam for p in probs], dtype=torch.float32, device="cuda")
    print("batching workload: one batched loss call", flush=True)
    g = fb.ctx.erbf_loss_grad_batched(fb.p, fb.m_dev, lambda_dev=lams, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    st = fb.ctx.stats()
    work = [p.levels[0].n ** 3 * p.m for p in probs]
    for b in (int(np.argmax(work)), int(np.argmin(work))):
        p = probs[b]
        print(f"batching workload: oracle of shape {b} ({p.levels[0].n}^3, {p.m} kernels)", flush=True)
        olv, _, _ = oracle_levels(p)
        K = O.kernels_from_packed(p.params, p.m, p.cap, p.cull_k)
        ref = pool.step(olv, K, mode=O.MODE_FIXED, lam=float(np.float32(p.lam)), tau1=TAU1, tau2=TAU2)
        a = _shape_grad(fb, g, b).astype(np.float64)[:, :p.m]
        gg = {"w": a[0], "c": a[1:4].T, "s": a[4:7].T, "q": a[7:11].T}
        go = oracle_grads_dict(ref.grads)
        errs = {k: rel_inf(gg[k], go[k]) for k in go}
        record(f"batching_config_shape{b}", n=p.levels[0].n, m=p.m, boundary_pairs=ref.n_amb,
               L2_rel=abs(st[b].L2 - ref.loss.L2) / ref.loss.L2, **errs)
        assert st[b].n_idall == ref.loss.n_idall
        assert abs(st[b].P_fwd - ref.P_fwd) <= ref.n_amb and abs(st[b].P_bwd - ref.P_bwd) <= ref.n_amb
        assert abs(st[b].L2 - ref.loss.L2) <= 1e-5 * ref.loss.L2
        for k in go:
            assert errs[k] <= 1e-4, (b, k, errs[k])
