"""Surface evaluation of Section 4 on the device against the oracle:
marching-tetrahedra triangles, area-uniform samples from the same uniforms,
HD / CD / CS of two point sets, the inverse of eq. 3-10, and the whole
pipeline on a synthetic shape (ground truth against an offset surface)."""

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import record
from oracle import metrics as Mx

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _shape_field(seed, n):
    prob = synth.make_custom(seed, [n], 8, (1.6, 2.6), kinds=("ellipsoid", "torus", "capsule"))
    lv = prob.levels[0]
    return lv.axis, lv.S


def test_extraction_matches_oracle():
    torch = _torch()
    from paper_2505_02350_amd import core
    for seed, n in ((91, 24), (92, 41)):
        ax, S = _shape_field(seed, n)
        dev = torch.device("cuda")
        T = core.erbf_surface_extract(torch.from_numpy(S).to(dev), n, torch.from_numpy(ax).to(dev), 0.0)
        torch.cuda.synchronize()
        ref = Mx.marching_tets(S, ax, 0.0)
        got = T.cpu().numpy().astype(np.float64)
        assert got.shape == ref.shape, (got.shape, ref.shape)
        err = float(np.abs(got - ref).max())
        record(f"surface_extract_{seed}", triangles=int(ref.shape[0]), err=err)
        assert err <= 2e-6


def test_capacity_error_and_retry():
    torch = _torch()
    from paper_2505_02350_amd import core, _lib as L
    ax, S = _shape_field(93, 20)
    dev = torch.device("cuda")
    with pytest.raises(L.ErbfError):
        core.erbf_surface_extract(torch.from_numpy(S).to(dev), 20, torch.from_numpy(ax).to(dev), 0.0, tri_cap=3)
    T = core.erbf_surface_extract(torch.from_numpy(S).to(dev), 20, torch.from_numpy(ax).to(dev), 0.0)
    assert T.shape[0] == Mx.marching_tets(S, ax).shape[0]


def test_sampling_matches_oracle():
    torch = _torch()
    from paper_2505_02350_amd import core
    ax, S = _shape_field(94, 32)
    tris = Mx.marching_tets(S, ax).astype(np.float32)
    u = np.random.default_rng(3).random((20000, 3)).astype(np.float32)
    dev = torch.device("cuda")
    P, N, W = core.erbf_surface_sample(torch.from_numpy(tris).to(dev), torch.from_numpy(u).to(dev))
    torch.cuda.synchronize()
    Pr, Nr, Wr = Mx.sample_surface(tris, u)
    same = float((W.cpu().numpy() == Wr).mean())
    e_p = float(np.abs(P.cpu().numpy() - Pr).max())
    e_n = float(np.abs(N.cpu().numpy() - Nr).max())
    record("surface_sample", same_triangle=same, e_p=e_p, e_n=e_n)
    assert same == 1.0 and e_p <= 1e-6 and e_n <= 1e-5


def test_metrics_match_oracle():
    torch = _torch()
    from paper_2505_02350_amd import core
    rng = np.random.default_rng(5)
    v = rng.normal(size=(30000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    w = rng.normal(size=(25000, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    Pt = (0.5 * v).astype(np.float32)
    Pr = (0.52 * w * (1 + 0.01 * rng.normal(size=(25000, 1)))).astype(np.float32)
    Nt, Nr = v.astype(np.float32), w.astype(np.float32)
    dev = torch.device("cuda")
    got = core.erbf_surface_metrics(*(torch.from_numpy(x).to(dev) for x in (Pt, Nt, Pr, Nr)))
    ref = Mx.surface_metrics(Pt, Nt, Pr, Nr)
    err = [abs(a - b) / abs(b) for a, b in zip(got, ref)]
    record("surface_metrics", got=got, ref=ref, err=err)
    assert max(err) <= 1e-5


def test_sdf_from_targets_matches_oracle():
    torch = _torch()
    from paper_2505_02350_amd import core
    ax, S = _shape_field(95, 24)
    m = O.sdf_min([S])
    t = O.targets_from_sdf(S, m).astype(np.float32)
    dev = torch.device("cuda")
    got = core.erbf_sdf_from_targets(torch.from_numpy(t).to(dev), float(np.float32(m))).cpu().numpy()
    ref = Mx.sdf_from_targets(t, float(np.float32(m)))
    assert np.allclose(got, ref.astype(np.float32), rtol=1e-6, atol=1e-7)


def test_pipeline_offset_surface():
    # ground truth S against S + 0.01 (an offset surface, 0.01 away): the
    # metrics are about (0.01, 0.01, 1) and match the oracle's pipeline
    torch = _torch()
    from paper_2505_02350_amd import core
    n = 48
    ax, S = _shape_field(96, n)
    Sr = (S.astype(np.float64) + 0.01).astype(np.float32)
    rng = np.random.default_rng(8)
    ut = rng.random((50000, 3)).astype(np.float32)
    ur = rng.random((50000, 3)).astype(np.float32)
    dev = torch.device("cuda")
    axd = torch.from_numpy(ax).to(dev)
    Tt = core.erbf_surface_extract(torch.from_numpy(S).to(dev), n, axd, 0.0)
    Tr = core.erbf_surface_extract(torch.from_numpy(Sr).to(dev), n, axd, 0.0)
    Pt, Nt, _ = core.erbf_surface_sample(Tt, torch.from_numpy(ut).to(dev))
    Pr, Nr, _ = core.erbf_surface_sample(Tr, torch.from_numpy(ur).to(dev))
    got = core.erbf_surface_metrics(Pt, Nt, Pr, Nr)
    rt = Mx.marching_tets(S, ax).astype(np.float32)
    rr = Mx.marching_tets(Sr, ax).astype(np.float32)
    qt = Mx.sample_surface(rt, ut)
    qr = Mx.sample_surface(rr, ur)
    ref = Mx.surface_metrics(qt[0].astype(np.float32), qt[1].astype(np.float32), qr[0].astype(np.float32),
                             qr[1].astype(np.float32))
    err = [abs(a - b) / abs(b) for a, b in zip(got, ref)]
    record("surface_pipeline", got=got, ref=ref, err=err)
    assert max(err) <= 1e-4
    assert 0.005 < got[1] < 0.02 and got[2] > 0.95


def test_extraction_with_infinite_values_matches_oracle():
    # the network's output taken back through eq. 3-10 is +inf where it is
    # <= 0: a field mixing finite and infinite values, as extracted by the oracle
    torch = _torch()
    from paper_2505_02350_amd import core
    ax, S = _shape_field(97, 20)
    F = S.copy()
    F[np.random.default_rng(2).random(F.size) < 0.2] = np.inf
    F[F > 0.3] = np.inf
    dev = torch.device("cuda")
    T = core.erbf_surface_extract(torch.from_numpy(F).to(dev), 20, torch.from_numpy(ax).to(dev), 0.0)
    torch.cuda.synchronize()
    ref = Mx.marching_tets(F, ax, 0.0)
    got = T.cpu().numpy().astype(np.float64)
    assert got.shape == ref.shape and np.all(np.isfinite(got))
    assert float(np.abs(got - ref).max()) <= 2e-6
