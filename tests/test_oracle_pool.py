"""The chunked, multi-process driver of the oracle gives the serial oracle's
step (sums over kernels regrouped, so equal to rounding)."""

import numpy as np

import oracle as O
from oracle import pool as oracle_pool
import synth


def test_pool_step_equals_serial_step():
    prob = synth.make_custom(31, [12, 20], 40, (1.6, 2.6), kinds=("ellipsoid", "box"), bands=[None, 0.2])
    S_all = [lv.S for lv in prob.levels]
    m = O.sdf_min(S_all)
    olv = [O.make_level(lv.n, lv.axis, active=lv.active_mask(),
                        t=O.targets_from_sdf(lv.S, m).astype(np.float32), S=lv.S) for lv in prob.levels]
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    ref = O.step(olv, K, mode=O.MODE_DYNAMIC, l1_active=True, tau_m=10.0)
    allow, n_amb = O.boundary_allowance(olv, K)
    for n_proc in (1, 3):
        got = oracle_pool.step(olv, K, mode=O.MODE_DYNAMIC, l1_active=True, tau_m=10.0, n_proc=n_proc)
        for a, b in zip(got.f, ref.f):
            assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
        for a, b in zip(got.allow, allow):
            assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
        assert got.n_amb == n_amb
        assert got.loss.n_idall == ref.loss.n_idall
        assert (got.P_fwd, got.P_bwd) == (ref.P_fwd, ref.P_bwd)
        assert abs(got.alpha - ref.alpha) < 1e-12
        for k in ("w", "c", "s", "q"):
            assert np.allclose(getattr(got.grads, k), getattr(ref.grads, k), rtol=1e-12, atol=1e-14)
