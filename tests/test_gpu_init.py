"""Inscribed-sphere initialisation on the device (Algorithm 1, eq. 3-11,
eq. 3-12) against the oracle: the chosen centres, their weights and the
uncovered count exactly, the eq. 3-12 scales to float rounding."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import GpuProblem, oracle_levels, record

pytestmark = pytest.mark.gpu

GAMMA = float(np.float32(1e-3))


def _init(prob, n_levels=None, max_centres=0, with_moments=False):
    lv, t32, _ = oracle_levels(prob)
    nl = len(lv) if n_levels is None else n_levels
    gp = GpuProblem(prob, t32, n_levels=nl)
    torch = gp.torch
    m1 = m2 = None
    if with_moments:
        m1 = torch.ones_like(gp.p)
        m2 = torch.ones_like(gp.p)
    nc, left = gp.ctx.erbf_init_inscribed(gp.p, gp.m_dev, 0, gamma=GAMMA, max_centres=max_centres, m1=m1, m2=m2)
    torch.cuda.synchronize()
    cap = prob.cap if max_centres <= 0 else min(max_centres, prob.cap)
    ref = O.inscribed_sphere_init(lv[:nl], gamma=GAMMA, m_max=cap)
    return gp, nc, left, ref, m1, m2


def _check(name, prob, gp, nc, left, ref):
    M = ref.index.size
    assert nc == M and int(gp.m_dev.item()) == M and left == ref.n_left, (nc, M, left, ref.n_left)
    P = gp.p.cpu().numpy().reshape(11, prob.cap)[:, :M].astype(np.float64)
    assert np.array_equal(P[0], ref.w)
    assert np.array_equal(P[1:4].T, ref.c)
    err_s = float(np.abs(P[4:7].T - ref.s).max()) if M else 0.0
    assert err_s <= 1e-6 * max(1.0, float(np.abs(ref.s).max()) if M else 1.0), err_s
    rot0 = 0.0 if prob.orientation == O.ORIENT_EULER else 1.0
    assert np.all(P[7] == rot0) and np.all(P[8:11] == 0.0)
    record(name, centres=M, left=left, err_s=err_s)


@pytest.mark.parametrize("orientation", [0, 1])
def test_init_matches_oracle_two_levels_with_band(orientation):
    prob = synth.make_custom(61, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus", "capsule"),
                             bands=[None, 0.2], cap=4096, orientation=orientation)
    gp, nc, left, ref, m1, m2 = _init(prob, with_moments=True)
    assert nc > 10
    _check(f"init_two_levels_o{orientation}", prob, gp, nc, left, ref)
    # the shape's moments are cleared
    assert float(m1.abs().max()) == 0.0 and float(m2.abs().max()) == 0.0


def test_init_centre_limit():
    prob = synth.make_custom(62, [24], 40, (1.6, 2.6), kinds=("ellipsoid",) * 4, cap=4096)
    gp, nc, left, ref, _, _ = _init(prob, max_centres=7)
    assert nc == 7 and left > 0
    _check("init_limit", prob, gp, nc, left, ref)


def test_init_single_centre_and_no_candidate():
    prob = synth.make_custom(63, [16], 40, (1.6, 2.6), kinds=("ellipsoid",), cap=64)
    gp, nc, left, ref, _, _ = _init(prob, max_centres=1)
    assert nc == 1 and ref.dhat[0] == 2.0
    _check("init_single", prob, gp, nc, left, ref)
    # targets with no interior point: no centre, m = 0
    torch = gp.torch
    lv, t32, _ = oracle_levels(prob)
    flat = np.full_like(t32[0], 0.5)
    gp2 = GpuProblem(prob, [flat])
    nc2, left2 = gp2.ctx.erbf_init_inscribed(gp2.p, gp2.m_dev, 0, gamma=GAMMA)
    torch.cuda.synchronize()
    assert nc2 == 0 and left2 == 0 and int(gp2.m_dev.item()) == 0


def test_init_full_size_starting_level():
    """The 64^3 starting level of the 64^3 -> 128^3 -> 256^3 workload
    (kernel capacity 16384): every centre exactly."""
    prob = synth.make_large()
    gp, nc, left, ref, _, _ = _init(prob, n_levels=1)
    assert nc > 1000 and left == 0
    _check("init_fullsize_64", prob, gp, nc, left, ref)


def test_init_full_size_two_levels_limited():
    """64^3 + 128^3 levels of the same workload, stopped after 2000 centres:
    the first 2000 centres and the uncovered count exactly."""
    prob = synth.make_large()
    gp, nc, left, ref, _, _ = _init(prob, n_levels=2, max_centres=2000)
    assert nc == 2000 and left > 0
    _check("init_fullsize_64_128_limit2000", prob, gp, nc, left, ref)


def test_init_then_forward_matches_oracle():
    """The initialised kernels feed the forward pass: the device field at the
    new parameters matches the oracle's on the same float32 parameters."""
    prob = synth.make_custom(64, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus"), cap=2048)
    gp, nc, left, ref, _, _ = _init(prob)
    torch = gp.torch
    f = torch.zeros(gp.ctx.n_points, dtype=torch.float32, device=gp.ctx.device)
    gp.ctx.erbf_loss_grad(gp.p, gp.m_dev, mode=O.MODE_FIXED, lam=0.0, f_out=f)
    torch.cuda.synchronize()
    lv, _, _ = oracle_levels(prob)
    K = O.kernels_from_packed(gp.p.cpu().numpy(), nc, prob.cap, prob.cull_k, prob.weight_map, prob.orientation)
    f_or = O.forward(lv, K)
    allow, _ = O.boundary_allowance(lv, K)
    fmax = max(np.abs(x).max() for x in f_or)
    worst = max(float((np.abs(fg.astype(np.float64) - fo) - al).max()) / fmax
                for fg, fo, al in zip(gp.split_points(f), f_or, allow))
    record("init_then_forward", centres=nc, e_f=worst, f_inf=fmax)
    assert worst <= 1e-5
