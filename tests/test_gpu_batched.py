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
    for v in (0, 1, 2, 3):
        print(f"batched loss_grad, 4 shapes, launch variant {v}", flush=True)
        fb.ctx.erbf_set_variant(v)
        g = fb.ctx.erbf_loss_grad_batched(fb.p, fb.m_dev, lambda_dev=lams, tau1=TAU1, tau2=TAU2)
        torch.cuda.synchronize()
        outs[v] = (g.clone(), fb.ctx.stats())
    for v in (1, 2, 3):
        assert torch.equal(outs[v][0], outs[0][0]), v
    gb, stb = outs[0]
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
    assert v in (0, 1, 2, 3) and fb.ctx.erbf_get_variant() == v
    assert all(t > 0 for t in times) and times[v] == min(times)
    assert torch.equal(fb.p, p0)
    g1 = fb.ctx.erbf_loss_grad(fb.p, fb.m_dev, lam=1e-4, tau1=TAU1, tau2=TAU2)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)
