"""Kernel timing (erbf_timing_enable / erbf_timing_read).

Every timed call is recorded; the forward, backward-tile and reduce
intervals are finite and non-negative, the backward's are positive, and
their sum stays within the wall time of the calls.  Cases: the plain step
(the backward's intervals start at the previous kernel's stop event), a step
with surface samples (sample kernels run in between, so the intervals take
their own start events), the fused forward + backward launch variant, and
the VJP (no forward).
"""

import math

import numpy as np
import pytest

import synth
from gpu_helpers import TAU1, TAU2, GpuProblem, oracle_levels

pytestmark = pytest.mark.gpu

N_CALLS = 4


def _timed(gp, call, tiles=True):
    torch = gp.torch
    gp.ctx.erbf_timing_enable(N_CALLS)
    call()   # the first call's events; the wall clock covers all of them
    torch.cuda.synchronize()
    gp.ctx.erbf_timing_read()
    gp.ctx.erbf_timing_enable(N_CALLS)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(N_CALLS):
        call()
    e1.record()
    torch.cuda.synchronize()
    wall = e0.elapsed_time(e1)
    f, b, r, n = gp.ctx.erbf_timing_read()
    print(f"forward {f:.4f} ms, backward tiles {b:.4f} ms, reduce {r:.4f} ms over {n} calls; wall {wall:.4f} ms",
          flush=True)
    assert n == N_CALLS
    for t in (f, b, r):
        assert math.isfinite(t) and t >= 0.0
    # (the fused variant's tile work is inside the forward's interval)
    assert r > 0.0 and (b > 0.0 or not tiles)
    assert f + b + r <= wall * 1.001 + 1e-3
    # the records are cleared by the read
    assert gp.ctx.erbf_timing_read()[3] == 0
    return f, b, r


def _gp(prob):
    _, t32, _ = oracle_levels(prob)
    return GpuProblem(prob, t32)


def _loss(gp):
    return lambda: gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, tau1=TAU1, tau2=TAU2, lam=1e-4)


def test_timing_of_the_step():
    gp = _gp(synth.make_custom(91, [24, 40], 300, (2.2, 3.0)))
    f, _, _ = _timed(gp, _loss(gp))
    assert f > 0.0


def test_timing_with_sample_kernels_in_between():
    prob = synth.make_custom(92, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus", "capsule"),
                             samples=(1, 3000, 32, 3010))
    gp = _gp(prob)
    f, _, _ = _timed(gp, _loss(gp))
    assert f > 0.0


def test_timing_of_the_fused_variant():
    gp = _gp(synth.make_custom(93, [24, 40], 300, (2.2, 3.0)))
    launch = gp.ctx.erbf_get_launch()
    launch["variant"] = 4
    gp.ctx.erbf_set_launch_dict(launch)
    f, _, _ = _timed(gp, _loss(gp), tiles=False)
    assert f > 0.0


def test_timing_of_the_vjp():
    torch = pytest.importorskip("torch")
    gp = _gp(synth.make_custom(94, [24, 40], 300, (2.2, 3.0)))
    rng = np.random.default_rng(5)
    up = torch.from_numpy(rng.standard_normal(gp.ctx.n_points).astype(np.float32)).to(gp.p.device)
    f, _, _ = _timed(gp, lambda: gp.ctx.erbf_vjp(gp.p, gp.m_dev, up))
    # no forward: two events recorded back to back (a few microseconds of
    # queue time each)
    assert f / N_CALLS < 0.01
