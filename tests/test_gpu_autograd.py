"""The autograd extension: ERBFField forward/backward through the C ABI,
checked against the oracle's vector-Jacobian product."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import GpuProblem, oracle_grads_dict, oracle_levels, record, rel_inf

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_autograd_matches_oracle_vjp():
    torch = _torch()
    from paper_2505_02350_amd.autograd import ERBFLayer
    prob = synth.make_custom(41, [16, 24], 30, (1.6, 2.6), kinds=("ellipsoid", "torus"), bands=[None, 0.2])
    olv, _, _ = oracle_levels(prob, with_targets=False)
    gp = GpuProblem(prob, None)
    layer = ERBFLayer(gp.ctx, gp.p, gp.m_dev)
    rng = np.random.default_rng(5)
    u = [rng.standard_normal(lv.npts).astype(np.float32) for lv in olv]
    ut = torch.from_numpy(np.concatenate(u)).to(gp.ctx.device)
    f = layer()
    loss = (f * ut).sum()
    loss.backward()
    torch.cuda.synchronize()
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    f_or = O.forward(olv, K)
    fg = np.concatenate(gp.split_points(f.detach()))
    assert np.abs(fg - np.concatenate(f_or)).max() <= 1e-5 * np.abs(np.concatenate(f_or)).max()
    # f is defined as 0 off the training mask, so the upstream is masked too
    gr = O.backward(olv, K, [np.where(lv.act(), uu.astype(np.float64), 0.0) for lv, uu in zip(olv, u)])
    gg = gp.grads_np(layer.p.grad)
    go = oracle_grads_dict(gr)
    errs = {k: rel_inf(gg[k], go[k]) for k in go}
    record("autograd_small", **errs)
    for k in go:
        assert errs[k] <= 1e-4, (k, errs[k])


def test_autograd_second_call_and_optimizer_step():
    torch = _torch()
    from paper_2505_02350_amd.autograd import ERBFLayer
    prob = synth.make_custom(42, [16], 20, (1.6, 2.6))
    gp = GpuProblem(prob, None)
    layer = ERBFLayer(gp.ctx, gp.p, gp.m_dev)
    opt = torch.optim.Adam(layer.parameters(), lr=1e-3)
    target = torch.zeros(gp.ctx.n_points, device=gp.ctx.device)
    losses = []
    for _ in range(3):
        opt.zero_grad()
        loss = ((layer() - target) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    # driving f towards zero must lower the loss
    assert losses[-1] < losses[0]
    # the backward holds no point-kernel pairs: the graph saved only p and m
    f = layer()
    assert f.grad_fn is not None and len(f.grad_fn.saved_tensors) == 2


def test_autograd_euler_orientation():
    torch = _torch()
    from paper_2505_02350_amd.autograd import ERBFLayer
    prob = synth.make_custom(43, [16, 24], 30, (1.6, 2.6), kinds=("ellipsoid", "torus"), bands=[None, 0.2],
                             orientation=1)
    olv, _, _ = oracle_levels(prob, with_targets=False)
    gp = GpuProblem(prob, None)
    layer = ERBFLayer(gp.ctx, gp.p, gp.m_dev)
    rng = np.random.default_rng(6)
    u = [rng.standard_normal(lv.npts).astype(np.float32) for lv in olv]
    (layer() * torch.from_numpy(np.concatenate(u)).to(gp.ctx.device)).sum().backward()
    torch.cuda.synchronize()
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k, 0, prob.orientation)
    gr = O.backward(olv, K, [np.where(lv.act(), uu.astype(np.float64), 0.0) for lv, uu in zip(olv, u)])
    gg = gp.grads_np(layer.p.grad)
    go = oracle_grads_dict(gr)
    errs = {k: rel_inf(gg[k], go[k]) for k in go}
    record("autograd_euler", **errs)
    for k in go:
        assert errs[k] <= 1e-4, (k, errs[k])
