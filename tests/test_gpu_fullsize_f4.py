"""Full-size parity of the widened rows on the 256^3 workload's data:

* octree layers 64^3 -> 128^3 -> 256^3 of the large shape, bit for bit;
* the snapshot step with 40 000 surface samples (the benchmark's --samples
  workload and launch configuration): f at 400 sampled samples against the
  oracle's per-point evaluation over all 16 384 kernels, and every sample's
  residual E = f - 1 consistent with it;
* the surface of the large shape's 128^3 signed distance: every triangle of
  marching tetrahedra against the oracle's.
"""

import numpy as np
import pytest

import oracle as O
import synth
from oracle import metrics as Mx
from gpu_helpers import record

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _torch():
    import torch
    return torch


def _bits_to_mask(bits, n):
    words = bits.cpu().numpy().view(np.uint32)
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:n].astype(bool)


def test_octree_layers_of_the_large_shape():
    torch = _torch()
    from paper_2505_02350_amd import core
    prob = synth.make_large()
    dev = torch.device("cuda")
    prev_bits, prev_mask = None, None
    counts = []
    for li in (1, 2):
        par = prob.levels[li - 1]
        S = torch.from_numpy(np.asarray(par.S, np.float32)).to(dev)
        bits = core.erbf_octree_bits(S, par.n, prev_bits)
        torch.cuda.synchronize()
        ref = O.octree_mask(par.S, par.n, prev_mask)
        got = _bits_to_mask(bits, (2 * par.n) ** 3)
        assert np.array_equal(got, ref), li
        counts.append(int(ref.sum()))
        prev_bits, prev_mask = bits, ref
    record("fullsize_octree", layers=[128, 256], active=counts)


def test_snapshot_with_40k_samples_sampled():
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    prob = synth.make_large_snapshot(samples=40000)
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=prob.cull_k, all_levels=True)
    f = torch.zeros(fit.ctx.n_points, dtype=torch.float32, device=fit.dev)
    G = torch.zeros_like(f)
    fit.ctx.erbf_loss_grad(fit.p, fit.m_dev, mode=L.MODE_DYNAMIC, l1_active=True, f_out=f, G_out=G,
                           tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)))
    torch.cuda.synchronize()
    st = fit.stats()[0]
    assert st.flags == 0
    base = fit.ctx.pt_base[0][3]
    P = prob.levels[3].samples
    fs = f[base:base + P.shape[0]].cpu().numpy().astype(np.float64)
    Gs = G[base:base + P.shape[0]].cpu().numpy().astype(np.float64)
    pick = np.random.default_rng(12).choice(P.shape[0], 400, replace=False)
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ref = O.forward_at_points(P[pick], K)
    allow, n_amb = O.allowance_at_points(P[pick], K)
    fmax = float(np.abs(ref).max())
    err = float((np.abs(fs[pick] - ref) - allow).max() / fmax)
    record("fullsize_samples_f", samples=400, e_f=err, f_inf=fmax, boundary_pairs=n_amb)
    assert err <= 1e-5
    # label 1: every sample is in id_all and carries G = 2 (f - 1)
    assert np.allclose(Gs, 2.0 * (fs - 1.0), rtol=0, atol=1e-6)


def test_surface_of_the_large_shape_at_128():
    torch = _torch()
    from paper_2505_02350_amd import core
    prob = synth.make_large()
    lv = prob.levels[1]
    dev = torch.device("cuda")
    T = core.erbf_surface_extract(torch.from_numpy(np.asarray(lv.S, np.float32)).to(dev), lv.n,
                                  torch.from_numpy(np.asarray(lv.axis, np.float32)).to(dev), 0.0)
    torch.cuda.synchronize()
    ref = Mx.marching_tets(lv.S, lv.axis, 0.0)
    got = T.cpu().numpy().astype(np.float64)
    assert got.shape == ref.shape
    err = float(np.abs(got - ref).max())
    record("fullsize_surface_128", triangles=int(ref.shape[0]), err=err)
    assert err <= 2e-6
