"""Pins for the oracle's reading of Algorithm 3's training control
(eq. l1_activate, eq. add_activate, eq. 3-27, the final phase)."""

import math

import numpy as np

from oracle import schedule as Sch


def _run(cfg, l2_seq, w_seq):
    st = Sch.ScheduleState(lr=cfg.lr0)
    out = []
    for l2, w in zip(l2_seq, w_seq):
        st = Sch.control_step(st, cfg, l2, np.asarray(w))
        out.append(st)
    return out


def test_l1_turns_on_when_the_l2_spread_settles():
    # alternating a, b has population std |a - b| / 2
    cfg = Sch.ScheduleConfig(k_l2=4, tau_l2=0.5, k_l1=1000)
    w = [np.ones(3)] * 12
    on = _run(cfg, [10.0, 10.9] * 6, w)            # std 0.45 < 0.5
    assert [s.l1_optim for s in on][:5] == [False, False, False, True, True]
    off = _run(cfg, [10.0, 11.1] * 6, w)           # std 0.55
    assert not any(s.l1_optim for s in off)


def test_adding_needs_stable_basis_count_and_switches_l1_off():
    cfg = Sch.ScheduleConfig(k_l2=2, tau_l2=1.0, k_l1=3, tau_l1=2.0, tau_d=0.01)
    ws = [np.array([0.5, 0.5, 0.5])] * 3 + [np.array([0.5, 0.5, 0.5, 0.5, 0.5, 0.5])] * 3
    st = _run(cfg, [5.0] * 6, ws)
    # e=2: L1 on (std 0); e=3: b_f window (3,3,3) -> add, L1 off; e=4: L1 on
    # again; b_f window (3,3,6) spread 3 -> no add; e=5 (3,6,6): no; e=6 (6,6,6): add
    assert [s.l1_optim for s in st] == [False, True, False, True, True, False]
    assert [s.add_request for s in st] == [False, False, True, False, False, True]
    assert [s.b_f for s in st] == [3, 3, 3, 6, 6, 6]


def test_pruning_epochs_and_effective_count_boundary():
    cfg = Sch.ScheduleConfig(k_l2=3, tau_l2=1.0, k_l1=1000, T_e=9, M_e=12, tau_d=0.01)
    w = np.array([0.01, -0.01, 0.0099, -0.2])
    assert Sch.effective_count(w, 0.01) == 3            # |w| = tau_d counts
    st = _run(cfg, [1.0] * 12, [w] * 12)
    # L1 on from e = 3 (after the check at e = 3); prune at e % 3 == 0 with L1 on and e < T_e
    assert [s.prune_now for s in st] == [False, False, False, False, False, True, False, False, False,
                                         False, False, False]
    assert st[8].final_phase and not st[8].l1_optim and not st[7].final_phase


def test_final_phase_cosine_learning_rate():
    cfg = Sch.ScheduleConfig(T_e=10, M_e=20, lr0=0.01, lr_final=1e-3, lr_min=1e-5)
    assert Sch.final_lr(cfg, 10) == 1e-3
    assert Sch.final_lr(cfg, 20) == 1e-5
    assert math.isclose(Sch.final_lr(cfg, 15), (1e-3 + 1e-5) / 2, rel_tol=1e-15)
    st = _run(cfg, [1.0] * 20, [np.ones(2)] * 20)
    assert all(s.lr == 0.01 for s in st[:9])
    assert st[9].final_phase and st[9].lr == Sch.final_lr(cfg, 11)


def test_refine_requests():
    cfg = Sch.ScheduleConfig(refine_epochs=(2, 5))
    st = _run(cfg, [1.0] * 6, [np.ones(2)] * 6)
    assert [s.refine_request for s in st] == [False, True, False, False, True, False]


def test_prune_is_a_stable_compaction():
    rng = np.random.default_rng(3)
    cap, m = 12, 9
    p = rng.normal(size=11 * cap)
    P = p.reshape(11, cap)
    P[0, :m] = [0.5, 0.001, -0.01, 0.02, -0.005, 0.3, 0.0, -0.7, 0.0099]
    m1 = rng.normal(size=11 * cap)
    new, nm, new_m1 = Sch.prune(p, m, cap, 0.01, m1)
    keep = [j for j in range(m) if abs(P[0, j]) >= 0.01]
    assert nm == len(keep) == 5
    N = new.reshape(11, cap)
    for k, j in enumerate(keep):
        assert np.array_equal(N[:, k], P[:, j])
        assert np.array_equal(new_m1.reshape(11, cap)[:, k], m1.reshape(11, cap)[:, j])
    assert not N[:, nm:].any()
