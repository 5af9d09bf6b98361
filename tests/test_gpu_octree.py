"""Octree layers on the device (eq. 3-16 on an octree, Section 3.4.2): the
layer masks bit for bit against the oracle, a full step on an octree
hierarchy, and the inscribed-sphere initialisation over its layers."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import GpuProblem, oracle_levels, record
from test_gpu_parity import _loss_case

pytestmark = pytest.mark.gpu


def _bits_to_mask(bits, n):
    words = bits.cpu().numpy().view(np.uint32)
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:n].astype(bool)


def test_octree_bits_match_oracle():
    import torch
    from paper_2505_02350_amd import core
    # ragged chain 12 -> 24 -> 48 and a power-of-two chain 8 -> 16 -> 32 -> 64
    for seed, ns in ((71, [12, 24, 48]), (72, [8, 16, 32, 64])):
        prob = synth.make_custom(seed, ns, 16, (1.6, 2.6), kinds=("ellipsoid", "torus", "box"),
                                 octree=[False] + [True] * (len(ns) - 1))
        lv, _, _ = oracle_levels(prob, with_targets=False)
        dev = torch.device("cuda")
        prev_bits = None
        counts = []
        for li in range(1, len(ns)):
            par = prob.levels[li - 1]
            S = torch.from_numpy(np.asarray(par.S, np.float32)).to(dev)
            bits = core.erbf_octree_bits(S, par.n, prev_bits)
            torch.cuda.synchronize()
            got = _bits_to_mask(bits, ns[li] ** 3)
            assert np.array_equal(got, lv[li].active), (seed, li)
            counts.append(int(got.sum()))
            prev_bits = bits
        record(f"octree_bits_{seed}", layers=ns, active=counts)


def test_step_on_octree_hierarchy():
    # 16^3 full, then two octree layers (32^3, 64^3); eq. 3-21 active
    prob = synth.make_custom(73, [16, 32, 64], 48, (1.8, 2.8), kinds=("ellipsoid", "torus", "capsule"),
                             octree=[False, True, True])
    _loss_case("loss_octree", prob, O.MODE_DYNAMIC, l1_active=True, tau_m=10.0)


def test_init_over_octree_layers():
    prob = synth.make_custom(74, [16, 32, 64], 48, (1.8, 2.8), kinds=("ellipsoid", "torus"),
                             octree=[False, True, True], cap=8192)
    lv, t32, _ = oracle_levels(prob)
    gp = GpuProblem(prob, t32)
    nc, left = gp.ctx.erbf_init_inscribed(gp.p, gp.m_dev, 0, gamma=float(np.float32(1e-3)))
    gp.torch.cuda.synchronize()
    ref = O.inscribed_sphere_init(lv, gamma=float(np.float32(1e-3)), m_max=prob.cap)
    assert nc == ref.index.size and left == ref.n_left
    P = gp.p.cpu().numpy().reshape(11, prob.cap)[:, :nc].astype(np.float64)
    assert np.array_equal(P[0], ref.w) and np.array_equal(P[1:4].T, ref.c)
    assert float(np.abs(P[4:7].T - ref.s).max()) <= 1e-6 * max(1.0, float(np.abs(ref.s).max()))
    record("init_octree", centres=nc, left=left)
