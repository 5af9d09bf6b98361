"""The method end to end on one synthetic shape through the library:
surface samples P with the first grid level, the inscribed-sphere
initialisation (Algorithm 1, nearest-sample depth), Algorithm 3's scheduled
training with a level appended on request, and the surface evaluation of
Section 4 before and after.  A property test: the loss falls and the fitted
zero set moves towards the true one."""

import numpy as np
import pytest

import synth
from gpu_helpers import record

pytestmark = pytest.mark.gpu


def test_init_schedule_and_evaluate():
    import torch
    from paper_2505_02350_amd import core
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    prob = synth.make_custom(101, [16, 32], 8, (2.0, 2.5), kinds=("ellipsoid", "torus"), cap=4096,
                             samples=(1, 3000, 16, 3000))
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=3.0, all_levels=False, pair_cap=1 << 22)
    fit.refine(0)            # 16^3
    fit.refine(0)            # the surface samples
    nc, left = fit.init_inscribed(0)
    assert nc > 10 and left == 0
    hd0, cd0, cs0 = fit.surface_metrics(0, 0, n_samples=20000, seed=1)
    cfg = core.sched_cfg(k_l2=5, tau_l2=1e6, k_l1=10, tau_l1=3.0, tau_d=0.01, T_e=150, M_e=200, lr0=1e-2,
                         lr_final=1e-3, lr_min=1e-5, refine_epochs=(60,))
    st, log = fit.fit_schedule(200, cfg, tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)), tau_m=1e3,
                               top_frac=0.01, k_new=64)
    torch.cuda.synchronize()
    hd1, cd1, cs1 = fit.surface_metrics(0, 0, n_samples=20000, seed=1)
    L2 = [r[0]["L2"] for r in log]
    record("pipeline", centres=nc, L2_first=L2[0], L2_last=L2[-1], m_last=log[-1][0]["m"],
           before=(hd0, cd0, cs0), after=(hd1, cd1, cs1), levels=fit.next_level[0])
    assert fit.next_level[0] == 3                      # the 32^3 level was appended
    assert all(np.isfinite(L2))
    assert cd1 < cd0 and cs1 > cs0
