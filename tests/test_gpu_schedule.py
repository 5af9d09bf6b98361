"""The device training control of Algorithm 3 (eq. l1_activate, eq.
add_activate, eq. 3-27, the final phase) against the oracle's reading, on
seeded synthetic inputs for two shapes at once, and a scheduled fit end to
end."""

import numpy as np
import pytest

import synth
from oracle import schedule as Sch

pytestmark = pytest.mark.gpu

F32 = lambda x: float(np.float32(x))  # noqa: E731  thresholds as the device holds them


def _torch():
    import torch
    return torch


def _write_l2(ctx, l2s):
    torch = _torch()
    from paper_2505_02350_amd import _lib as L
    arr = (L.Stats * ctx.n_shapes)()
    for b, v in enumerate(l2s):
        arr[b].L2 = v
    ctx.stats_buf.copy_(torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(ctx.device))


def test_control_matches_oracle_on_synthetic_inputs():
    torch = _torch()
    from paper_2505_02350_amd import core
    caps = [40, 30]
    ctx = core.Context([([8], caps[0]), ([8], caps[1])], 4096, 3.0)
    ax = torch.from_numpy(synth.axis_coords(8)).to(ctx.device)
    for b in range(2):
        ctx.erbf_refine_level(b, ax)
    kw = dict(k_l2=3, tau_l2=0.6, k_l1=4, tau_l1=2.0, tau_d=0.05, T_e=25, M_e=30, lr0=0.01, lr_final=1e-3,
              lr_min=1e-5, refine_epochs=(5, 12))
    cfg = core.sched_cfg(**kw)
    ocfg = Sch.ScheduleConfig(**{k: (F32(v) if isinstance(v, float) else v) for k, v in kw.items()})
    st = core.SchedState(ctx, cfg)
    ctx.erbf_sched_init(cfg, st)
    ost = [Sch.ScheduleState(lr=ocfg.lr0) for _ in range(2)]
    rng = np.random.default_rng(77)
    C = ctx.cap_total
    m = [30, 22]
    seen = {"prune": 0, "add": 0, "l1": 0, "final": 0, "refine": 0}
    for e in range(1, 31):
        # L2: shape 0 settles at once (std 0.2), shape 1 only after step 14
        l2 = [10.0 + 0.2 * (-1) ** e, 10.0 + (1.0 * (-1) ** e if e <= 14 else 0.0)]
        # weights: a few effective ones, the rest below tau_d; moments random
        p = rng.normal(size=11 * C).astype(np.float32)
        m1 = rng.normal(size=11 * C).astype(np.float32)
        m2 = rng.random(size=11 * C).astype(np.float32)
        P = p.reshape(11, C)
        for b, kb in enumerate((0, caps[0])):
            # the effective count swings by 3 until step 16, then holds
            n_eff = [8, 6][b] + (3 if (e % 2 and e < 16) else 0)
            w = np.full(m[b], 0.01, np.float32)
            w[rng.permutation(m[b] - 1)[:n_eff]] = 0.5
            w[m[b] - 1] = np.float32(0.05)            # exactly tau_d: effective, kept
            P[0, kb:kb + m[b]] = w * np.where(rng.random(m[b]) < 0.5, -1, 1)
        dev = ctx.device
        pt = torch.from_numpy(p).to(dev)
        m1t = torch.from_numpy(m1).to(dev)
        m2t = torch.from_numpy(m2).to(dev)
        m_dev = torch.tensor(m, dtype=torch.int32, device=dev)
        _write_l2(ctx, l2)
        ctx.erbf_sched_step(pt, m_dev, cfg, st, m1t, m2t)
        torch.cuda.synchronize()
        pg, m1g, m2g, mg = pt.cpu().numpy().reshape(11, C), m1t.cpu().numpy(), m2t.cpu().numpy(), m_dev.cpu().tolist()
        for b, kb in enumerate((0, caps[0])):
            cap = caps[b]
            seg = P[:, kb:kb + cap].reshape(-1)
            ost[b] = Sch.control_step(ost[b], ocfg, l2[b], seg.reshape(11, cap)[0, :m[b]])
            o = ost[b]
            got = dict(epoch=int(st.epoch[b]), l1=bool(st.l1_active[b]), fin=bool(st.final_phase[b]),
                       add=bool(st.add_request[b]), ref=bool(st.refine_request[b]), bf=int(st.b_f[b]))
            want = dict(epoch=o.epoch, l1=o.l1_optim, fin=o.final_phase, add=o.add_request, ref=o.refine_request,
                        bf=o.b_f)
            assert got == want, (e, b, got, want)
            assert abs(float(st.lr[b]) - o.lr) <= 1e-6 * o.lr
            if o.prune_now:
                seen["prune"] += 1
                m1s = m1.reshape(11, C)[:, kb:kb + cap].reshape(-1)
                m2s = m2.reshape(11, C)[:, kb:kb + cap].reshape(-1)
                newp, nm, n1, n2 = Sch.prune(seg, m[b], cap, ocfg.tau_d, m1s, m2s)
                assert mg[b] == nm and int(st.n_pruned[b]) == m[b] - nm
                assert np.array_equal(pg[:, kb:kb + nm], newp.reshape(11, cap)[:, :nm].astype(np.float32))
                assert np.array_equal(m1g.reshape(11, C)[:, kb:kb + m[b]], n1.reshape(11, cap)[:, :m[b]])
                assert np.array_equal(m2g.reshape(11, C)[:, kb:kb + m[b]], n2.reshape(11, cap)[:, :m[b]])
                m[b] = nm
            else:
                assert mg[b] == m[b] and int(st.n_pruned[b]) == 0
                assert np.array_equal(pg[:, kb:kb + cap], P[:, kb:kb + cap])
            seen["add"] += o.add_request
            seen["l1"] += o.l1_optim
            seen["final"] += o.final_phase
            seen["refine"] += o.refine_request
    # every branch of the control was taken
    assert all(v > 0 for v in seen.values()), seen


def _scheduled_fit():
    torch = _torch()
    from paper_2505_02350_amd import core
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    prob = synth.make_custom(57, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus"), bands=[None, 0.15],
                             cap=200)
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=3.0, all_levels=False)
    fit.refine(0)
    cfg = core.sched_cfg(k_l2=4, tau_l2=1e6, k_l1=6, tau_l1=3.0, tau_d=0.02, T_e=40, M_e=50, lr0=1e-2,
                         lr_final=1e-3, lr_min=1e-5, refine_epochs=(10,))
    st, log = fit.fit_schedule(50, cfg, tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)), tau_m=1e3,
                               top_frac=0.05, k_new=16)
    torch.cuda.synchronize()
    return fit, st, log


def test_scheduled_fit_takes_every_branch_and_is_deterministic():
    torch = _torch()
    fit, st, log = _scheduled_fit()
    rows = [r[0] for r in log]
    assert fit.next_level[0] == 2                          # the level request was served
    assert any(r["n_added"] > 0 for r in rows)             # eq. add_activate fired and Algorithm 2 ran
    assert any(r["n_pruned"] > 0 for r in rows)            # eq. 3-27 removed kernels
    assert any(r["l1"] for r in rows) and not rows[-1]["l1"]
    assert int(st.final_phase[0]) == 1 and abs(float(st.lr[0]) - 1e-5) < 1e-9
    assert all(np.isfinite(r["L2"]) for r in rows)
    fit2, _, log2 = _scheduled_fit()
    assert torch.equal(fit.p, fit2.p) and torch.equal(fit.m_dev, fit2.m_dev)
    assert [r[0]["L2"] for r in log2] == [r["L2"] for r in rows]


def test_checkpoint_resume_continues_bit_for_bit(tmp_path):
    """A scheduled fit saved after 25 steps (past a seeding and the level
    request) and resumed in a fresh context for 25 more steps ends with the
    same parameters, counts and per-step L2 as one run of 50 steps; the
    JSON-lines log holds one row per step."""
    import json
    torch = _torch()
    from paper_2505_02350_amd import core
    from paper_2505_02350_amd.fit import Fitter, ShapeInput, jsonl_logger
    prob = synth.make_custom(57, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus"), bands=[None, 0.15],
                             cap=200)
    cfg = core.sched_cfg(k_l2=4, tau_l2=1e6, k_l1=6, tau_l1=3.0, tau_d=0.02, T_e=40, M_e=50, lr0=1e-2,
                         lr_final=1e-3, lr_min=1e-5, refine_epochs=(10,))
    kw = dict(tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)), tau_m=1e3, top_frac=0.05, k_new=16)

    def new_fit():
        f = Fitter([ShapeInput.from_problem(prob)], cull_k=3.0, all_levels=False)
        f.refine(0)
        return f

    print("scheduled fit: 50 steps in one run", flush=True)
    full = new_fit()
    _, log_full = full.fit_schedule(50, cfg, **kw)
    print("scheduled fit: 25 steps, checkpoint, 25 more in a fresh context", flush=True)
    first = new_fit()
    st, log_a = first.fit_schedule(25, cfg, on_step=jsonl_logger(str(tmp_path / "log.jsonl")), **kw)
    ck = str(tmp_path / "ck.npz")
    first.save(ck, st)
    del first
    second = new_fit()
    st2 = core.SchedState(second.ctx, cfg)
    second.load(ck, st2)
    _, log_b = second.fit_schedule(25, cfg, state=st2, **kw)
    torch.cuda.synchronize()
    assert second.next_level[0] == 2
    assert any(r[0]["n_added"] > 0 for r in log_a)
    assert torch.equal(full.p, second.p) and torch.equal(full.m_dev, second.m_dev)
    assert torch.equal(full.m1, second.m1) and torch.equal(full.step_dev, second.step_dev)
    assert [r[0]["L2"] for r in log_full] == [r[0]["L2"] for r in log_a + log_b]
    rows = [json.loads(x) for x in open(tmp_path / "log.jsonl")]
    assert [r["step"] for r in rows] == list(range(25)) and rows[-1]["shapes"][0]["L2"] == log_a[-1][0]["L2"]


def test_lagged_fit_matches_waiting_fit_bit_for_bit():
    """The scheduled fit that enqueues each step before reading the previous
    one (the control's hold word voids the step after a request, which is
    then taken again) follows the same trajectory as the fit that waits for
    every step: two shapes whose requests come at different steps, growth
    rounds, a level request, pruning; parameters, moments, counters, control
    state and every log row equal."""
    torch = _torch()
    from paper_2505_02350_amd import core
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    probs = [synth.make_custom(57, [16, 24], 40, (1.6, 2.6), kinds=("ellipsoid", "torus"), bands=[None, 0.15],
                               cap=200),
             synth.make_custom(61, [16, 24], 48, (1.4, 2.4), kinds=("box", "ellipsoid"), bands=[None, 0.15],
                               cap=160)]
    cfg = core.sched_cfg(k_l2=4, tau_l2=1e6, k_l1=6, tau_l1=3.0, tau_d=0.02, T_e=40, M_e=50, lr0=1e-2,
                         lr_final=1e-3, lr_min=1e-5, refine_epochs=(10,))
    kw = dict(tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)), tau_m=1e3, top_frac=0.05, k_new=16,
              add_every=9)
    runs = []
    for lagged in (False, True):
        print(f"scheduled fit, two shapes, lagged={lagged}", flush=True)
        f = Fitter([ShapeInput.from_problem(p) for p in probs], cull_k=3.0, all_levels=False)
        f.refine(0)
        f.refine(1)
        st, log = f.fit_schedule(50, cfg, lagged=lagged, **kw)
        torch.cuda.synchronize()
        runs.append((f, st, log))
    (fa, sa, la), (fb, sb, lb) = runs
    assert la == lb
    assert sum(r[b]["n_added"] > 0 for r in la for b in range(2)) >= 3
    assert any(r[b]["n_pruned"] > 0 for r in la for b in range(2))
    assert fa.next_level == fb.next_level == [2, 2]
    for name in ("p", "m_dev", "m1", "m2", "step_dev"):
        assert torch.equal(getattr(fa, name), getattr(fb, name)), name
    for name in ("flags", "lr", "l2_ring", "bf_ring"):
        assert torch.equal(getattr(sa, name), getattr(sb, name)), name
    assert int(sb.hold[0]) == 0
