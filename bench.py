#!/usr/bin/env python3
"""Benchmark of one SE-RBFNet optimisation step on the MI355X.

Workload (timing snapshot of the large hierarchy): smooth union of 12 boxes,
6 capsules and 4 tori sampled on 64^3 + 128^3 + 256^3 grid levels (the finest
restricted to |S| < 0.1), 16384 ERBFs drawn with the kernel init rule.  One
step = kernel records and tile buckets, forward + masked loss, backward, eq. 3-21
weights and Adam, all on the device; inputs are resident in HBM before the
timed region.

Prints one JSON line.  `value` is whole-step pair throughput,
(P_fwd + P_bwd) per step divided by the wall time of a step.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FWD_FLOP_PER_PAIR = 25.0   # delta 3, ball test 5, quadric 14, exp2 1, accumulate 2
BWD_FLOP_PER_PAIR = 43.0   # + g 1, T0 1, g*delta 3, T1 3, T2 12
FP32_VECTOR_PEAK = 157.3e12
COPY_CAL_BYTES = 256 * 1024 * 1024
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_large_snapshot.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def under_profiler() -> bool:
    """True when a profiler's tool library is preloaded into this process: then
    nothing here forks (children would inherit the profiler's session)."""
    env = os.environ
    return "rocprof" in env.get("LD_PRELOAD", "") or any(k.startswith("ROCPROF") for k in env)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, n_proc):
    """The FP64 oracle's culled forward + loss + backward + eq. 3-21 weights
    over the whole workload (every kernel, every point of the three levels),
    its kernels split over `n_proc` worker processes, timed on the host."""
    from oracle import erbf as O
    from oracle import pool
    S_all = [lv.S for lv in prob.levels]
    m = O.sdf_min(S_all)
    olv = [O.make_level(lv.n, lv.axis, active=(O.band_mask(lv.S, lv.band) if lv.band else None),
                        t=O.targets_from_sdf(lv.S, m).astype(np.float32), S=lv.S) for lv in prob.levels]
    K = O.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k)
    t0 = time.perf_counter()
    ref = pool.step(olv, K, mode=O.MODE_DYNAMIC, l1_active=True, tau1=float(np.float32(0.9)),
                    tau2=float(np.float32(1.1)), tau_m=float(np.float32(0.02)), n_proc=n_proc)
    dt = time.perf_counter() - t0
    pairs = ref.P_fwd + ref.P_bwd
    return {"value": pairs / dt, "unit": "pairs/s", "cores": n_proc, "kind": "oracle",
            "sample": f"the whole first step of the workload ({prob.m} kernels, all 3 levels): culled fwd + loss + "
                      f"bwd + eq. 3-21 in float64 numpy over {n_proc} worker processes, {dt:.1f} s, {pairs} pairs",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def batching_bench(probs, steps, warmup):
    """64 shapes (grids 32^3..128^3, 256..4096 kernels, per-shape lambda):
    one batched context with a HIP-graph step vs 64 plain contexts, each with
    its own graph, replayed one after another.  Aggregate pair throughput."""
    import torch
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd.fit import Fitter, ShapeInput

    shapes = [ShapeInput.from_problem(p) for p in probs]
    lams = [p.lam for p in probs]
    kw = dict(mode=L.MODE_FIXED, lr=1e-3)

    fb = Fitter(shapes, cull_k=3.0)
    lam_dev = torch.tensor(lams, dtype=torch.float32, device=fb.dev)
    fb.ctx.erbf_autotune(fb.p, fb.m_dev, reps=2, lambda_dev=lam_dev)
    launch_b = fb.ctx.erbf_get_launch()
    # equal accuracy: the first step's gradients are bitwise those of the plain fits
    gb = fb.ctx.erbf_loss_grad_batched(fb.p, fb.m_dev, lambda_dev=lam_dev).clone()
    # the plain fits: one launch choice per grid-size class, tuned on the
    # class's first shape and kept by every context of the class
    per_class = {}
    plains = []
    for b, s in enumerate(shapes):
        f = Fitter([s], cull_k=3.0)
        cls = str(s.level_ns[0])
        if cls not in per_class:
            f.ctx.erbf_autotune(f.p, f.m_dev, reps=2, lam=lams[b])
            per_class[cls] = f.ctx.erbf_get_launch()
        else:
            f.ctx.erbf_set_launch_dict(per_class[cls])
        g = f.ctx.erbf_loss_grad(f.p, f.m_dev, lam=lams[b])
        kb, cap = fb.ctx.kbase[b], s.cap
        same = torch.equal(gb.view(11, -1)[:, kb:kb + cap], g.view(11, -1)[:, :cap])
        if not same:
            raise SystemExit(f"batched and plain gradients differ for shape {b}")
        plains.append(f)
    torch.cuda.synchronize()

    fb.capture(lambda_dev=lam_dev, **kw)
    for f, lam in zip(plains, lams):
        f.capture(lam=lam, **kw)
    for _ in range(warmup):
        fb.replay()
        for f in plains:
            f.replay()
    torch.cuda.synchronize()

    fb.ctx.reset_stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        fb.replay()
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    pairs_b = sum(st.P_fwd_total + st.P_bwd_total for st in fb.stats())

    for f in plains:
        f.ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in plains:
        for _ in range(steps):
            f.replay()
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    pairs_p = sum(f.stats()[0].P_fwd_total + f.stats()[0].P_bwd_total for f in plains)
    thr_b, thr_p = pairs_b / wall_b, pairs_p / wall_p
    log(f"batched {1e3 * wall_b / steps:.2f} ms/step, plain {1e3 * wall_p / steps:.2f} ms per step of all shapes")
    return {
        "workload": "64 shapes: smooth unions of 2-10 ellipsoids/tori on 32^3..128^3 grids, 256..4096 ERBFs, "
                    "per-shape lambda, seed 3",
        "points": int(sum(p.levels[0].n ** 3 for p in probs)),
        "kernels": int(sum(p.m for p in probs)),
        "steps": steps,
        "batched_ms_per_step": 1e3 * wall_b / steps,
        "plain_ms_per_step_all_shapes": 1e3 * wall_p / steps,
        "batched_pairs_per_s": thr_b,
        "plain_pairs_per_s": thr_p,
        "speedup": thr_b / thr_p,
        "launch_batched": launch_b,
        "launch_plain_per_grid_class": dict(sorted(per_class.items(), key=lambda kv: int(kv[0]))),
        "equal_accuracy": "first-step gradients bitwise equal to the plain fits",
    }


def init_bench(reps=3, with_cpu=True):
    """Inscribed-sphere initialisation (Algorithm 1, eq. 3-11/3-12) of the
    large workload's shape on its 64^3 starting level, then on 64^3 + 128^3
    (kernel capacity 16384).  Each call is synchronous; the figure is the
    median wall time of `reps` calls after one untimed call."""
    import torch
    import synth
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    prob = synth.make_large()
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=prob.cull_k, all_levels=False)
    rows = []
    for nl in (1, 2):
        fit.refine(0)
        times = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nc, left = fit.ctx.erbf_init_inscribed(fit.p, fit.m_dev, 0, gamma=1e-3, m1=fit.m1, m2=fit.m2)
            times.append(time.perf_counter() - t0)
        ms = 1e3 * float(np.median(times[1:]))
        interior = int(sum(np.count_nonzero(lv.S < 0) for lv in prob.levels[:nl]))
        rows.append({"levels": "+".join(f"{lv.n}^3" for lv in prob.levels[:nl]), "points_S_negative": interior,
                     "centres": nc, "uncovered": left, "ms": ms, "us_per_round": 1e3 * ms / (nc + 1)})
        log(f"inscribed-sphere init on {rows[-1]['levels']}: {nc} centres, {left} uncovered, {ms:.2f} ms")
    out = {"workload": "large: shape of seed 2 (12 boxes + 6 capsules + 4 tori), gamma 1e-3, capacity 16384",
           "runs": rows}
    if with_cpu:
        import oracle as O
        S_all = [lv.S for lv in prob.levels]
        msdf = O.sdf_min(S_all)
        lv0 = prob.levels[0]
        olv = O.make_level(lv0.n, lv0.axis, t=O.targets_from_sdf(lv0.S, msdf).astype(np.float32), S=lv0.S)
        t0 = time.perf_counter()
        ref = O.inscribed_sphere_init([olv], gamma=float(np.float32(1e-3)), m_max=prob.cap)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1e3 * cpu_s, "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"the whole 64^3 initialisation ({ref.index.size} centres)"}
    return out


def minibatch_bench(steps, warmup, batch=10000):
    """Mini-batch steps of Algorithm 3 (B_s = 10000 points per batch, loss +
    gradient + Adam) on the large snapshot workload, batches drawn from one
    seeded permutation of its training points."""
    import torch
    import synth
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    prob = synth.make_large_snapshot()
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=prob.cull_k, all_levels=True, batch_cap=batch)
    pts = fit.training_points(0)
    order = torch.from_numpy(pts[np.random.default_rng(0).permutation(pts.size)]).to(fit.dev)
    nb = pts.size // batch

    def one(i):
        idx = order[(i % nb) * batch:(i % nb + 1) * batch]
        fit.ctx.erbf_loss_grad_minibatch(fit.p, fit.m_dev, idx, mode=L.MODE_DYNAMIC, l1_active=True, grad_out=fit.grad)
        fit.ctx.erbf_adam_step(fit.p, fit.m_dev, fit.grad, fit.m1, fit.m2, fit.step_dev, lr=prob.lr)

    for i in range(warmup):
        one(i)
    torch.cuda.synchronize()
    fit.ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one(warmup + i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = fit.stats()[0]
    ms = 1e3 * wall / steps
    log(f"mini-batch: {ms:.3f} ms per batch of {batch}")
    return {"workload": "large_snapshot, batches of 10000 training points (seeded permutation)",
            "batch": batch, "steps": steps, "ms_per_batch": ms,
            "pairs_per_s": (st.P_fwd_total + st.P_bwd_total) / wall,
            "batches_per_epoch": int(-(-pts.size // batch)),
            "ms_per_epoch": ms * (-(-pts.size // batch))}


def variant_bench(kind, steps, warmup):
    """The step on a variant of the large snapshot: octree layers in place of
    the band (kind "octree"), or the snapshot plus 40 000 surface samples
    (kind "samples", the paper's sample count)."""
    import torch
    import synth
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    if kind == "octree":
        prob = synth.make_large_snapshot(octree=True)
        what = "64^3 + octree layers 128^3, 256^3 (parent |S| <= half-diagonal), 16384 ERBFs, seed 2"
    else:
        prob = synth.make_large_snapshot(samples=40000)
        what = "large_snapshot + 40000 surface samples (label 1) binned on 64^3 cells, 16384 ERBFs, seed 2"
    fit = Fitter([ShapeInput.from_problem(prob)], cull_k=prob.cull_k, all_levels=True)
    kw = dict(mode=L.MODE_DYNAMIC, l1_active=True, lr=prob.lr)
    for _ in range(warmup):
        fit.step(**kw)
    torch.cuda.synchronize()
    fit.ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fit.step(**kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = fit.stats()[0]
    if st.flags:
        raise SystemExit(f"{kind}: bucket overflow")
    pts = int(fit.training_points(0).size)
    log(f"{kind}: {1e3 * wall / steps:.3f} ms/step over {pts} training points")
    return {"workload": what, "training_points": pts, "steps": steps, "ms_per_step": 1e3 * wall / steps,
            "pairs_per_s": (st.P_fwd_total + st.P_bwd_total) / wall,
            "P_fwd_per_step": st.P_fwd_total / steps, "P_bwd_per_step": st.P_bwd_total / steps}


def surface_bench(n_samples=100000, with_cpu=True):
    """Surface evaluation of Section 4 at the paper's sample count: the zero
    set of the large workload's 256^3 signed distance against that of a
    stand-in reconstruction (the field sent through eq. 3-10 and back, moved
    by 0.004), each extracted by marching tetrahedra, 10^5 area-uniform
    samples each (seeded uniforms), then HD / CD / CS."""
    import torch
    import synth
    from paper_2505_02350_amd import core
    prob = synth.make_large()
    lv = prob.levels[2]
    n = lv.n
    dev = torch.device("cuda")
    ax = torch.from_numpy(np.asarray(lv.axis, np.float32)).to(dev)
    S = torch.from_numpy(np.asarray(lv.S, np.float32)).to(dev)
    m = float(np.float32(min(float(np.min(l.S)) for l in prob.levels)))
    t = core.erbf_targets_from_sdf(S, m)
    Sr = core.erbf_sdf_from_targets(t, m) + 0.004
    rng = np.random.default_rng(17)
    ut = torch.from_numpy(rng.random((n_samples, 3)).astype(np.float32)).to(dev)
    ur = torch.from_numpy(rng.random((n_samples, 3)).astype(np.float32)).to(dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t0)

    core.erbf_surface_extract(S, n, ax, 0.0)   # warm-up (module load, allocator)
    Tt, ms_et = timed(lambda: core.erbf_surface_extract(S, n, ax, 0.0, tri_cap=4 * n * n * 6))
    Tr, ms_er = timed(lambda: core.erbf_surface_extract(Sr, n, ax, 0.0, tri_cap=4 * n * n * 6))
    (Pt, Nt, _), ms_st = timed(lambda: core.erbf_surface_sample(Tt, ut))
    (Pr, Nr, _), ms_sr = timed(lambda: core.erbf_surface_sample(Tr, ur))
    (hd, cd, cs), ms_m = timed(lambda: core.erbf_surface_metrics(Pt, Nt, Pr, Nr))
    log(f"surface: {Tt.shape[0]} / {Tr.shape[0]} triangles, extract {ms_et:.1f} ms, sample {ms_st:.1f} ms, "
        f"metrics {ms_m:.1f} ms; HD {hd:.4g} CD {cd:.4g} CS {cs:.6f}")
    out = {"workload": "large (seed 2) 256^3 signed distance vs the same through eq. 3-10 and back, moved by 0.004; "
                       f"{n_samples} samples per surface",
           "triangles": [int(Tt.shape[0]), int(Tr.shape[0])], "extract_ms": [ms_et, ms_er],
           "sample_ms": [ms_st, ms_sr], "metrics_ms": ms_m, "pairs_per_s_metrics": 2.0 * n_samples * n_samples /
           (ms_m * 1e-3), "HD": hd, "CD": cd, "CS": cs}
    if with_cpu:
        from oracle import metrics as Mx
        a = [x.cpu().numpy() for x in (Pt, Nt, Pr, Nr)]
        t0 = time.perf_counter()
        ref = Mx.surface_metrics(*a)
        out["cpu_baseline"] = {"value": 1e3 * (time.perf_counter() - t0), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": "the metrics stage on the same point sets (k-d trees)",
                               "metrics": list(ref)}
    return out


def autograd_steps(fit, steps):
    """Steps through the differentiable field (forward erbf_eval, backward
    erbf_vjp recomputing the responses) with a squared-residual loss on the
    first level's targets and torch's Adam; ms per step."""
    import torch
    from paper_2505_02350_amd.autograd import ERBFLayer
    layer = ERBFLayer(fit.ctx, fit.p, fit.m_dev)
    t = fit._levels[0][1]
    opt = torch.optim.Adam(layer.parameters(), lr=1e-4)
    for i in range(steps + 2):
        if i == 2:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        opt.zero_grad(set_to_none=False)
        f = layer()
        loss = ((f[:t.numel()] - t) ** 2).sum()
        loss.backward()
        opt.step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    log(f"autograd layer: {ms:.3f} ms per step, loss {float(loss):.4g}")
    return {"steps": steps, "ms_per_step": ms, "loss_last": float(loss)}


def e2e_bench(name, prob=None):
    """One of the benchmark configurations run end to end: the whole training loop
    on the device (the fixed-weight loop of the tiny config; Algorithm 3's
    control with eq. 3-21, pruning, kernel addition and level appends for
    mid, large and diff; 200 batched steps against 64 sequential plain fits
    for batching), then Section 4's HD / CD / CS of the result against the
    ground-truth zero set on the finest grid level (10^5 samples each)."""
    import torch
    import synth
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd import core
    from paper_2505_02350_amd.fit import Fitter, ShapeInput
    tau = dict(tau1=float(np.float32(0.9)), tau2=float(np.float32(1.1)), tau_m=float(np.float32(0.02)))
    t_gen = time.perf_counter()
    if name == "batching":
        probs = synth.make_batching()
        log(f"{name}: workload generated in {time.perf_counter() - t_gen:.1f} s")
        shapes = [ShapeInput.from_problem(p) for p in probs]
        lams = torch.tensor([p.lam for p in probs], dtype=torch.float32)
        fb = Fitter(shapes, cull_k=3.0)
        kw = dict(mode=L.MODE_FIXED, lr=1e-3, **tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(200):
            fb.step(lambda_dev=lams.to(fb.dev), **kw)
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t0
        L2b = [st.L2 for st in fb.stats()]
        del fb
        torch.cuda.empty_cache()
        wall_p, L2p = 0.0, []
        for b, sh in enumerate(shapes):
            f = Fitter([sh], cull_k=3.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(200):
                f.step(lam=float(lams[b]), **kw)
            torch.cuda.synchronize()
            wall_p += time.perf_counter() - t0
            L2p.append(f.stats()[0].L2)
            del f
        rel = max(abs(a - b) / max(abs(b), 1e-300) for a, b in zip(L2b, L2p))
        log(f"{name}: 200 steps batched {wall_b:.2f} s, 64 plain fits {wall_p:.2f} s, final L2 rel diff {rel:.3g}")
        return {"config": name, "steps": 200, "batched_s": wall_b, "plain_s": wall_p, "speedup": wall_p / wall_b,
                "final_L2_max_rel_diff": rel}
    if prob is not None:
        pass
    elif name == "tiny":
        prob = synth.make_tiny()
    elif name == "mid":
        prob = synth.make_mid()
    elif name in ("large", "large-growth"):
        prob = synth.make_large()
    elif name == "diff":
        prob = synth.make_diff()
    else:
        raise SystemExit(f"unknown e2e config {name}")
    log(f"{name}: workload generated in {time.perf_counter() - t_gen:.1f} s")
    shape = ShapeInput.from_problem(prob)
    hier = name.startswith("large")
    # list capacity for kernels of any scale the run may add (eq. 3-24 floors
    # the scale at the finest grid spacing)
    pair_cap = {"tiny": 1 << 20, "mid": 1 << 26, "diff": 1 << 27}.get(name, 1 << 26)
    fit = Fitter([shape], cull_k=prob.cull_k, pair_cap=pair_cap, all_levels=not hier)
    if hier:
        fit.refine(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if name == "tiny":
        steps = 100
        for _ in range(steps):
            fit.step(mode=L.MODE_FIXED, lam=prob.lam, lr=prob.lr, **tau)
        torch.cuda.synchronize()
        n_add = n_prune = 0
    else:
        steps = {"mid": 500, "diff": 2000}.get(name, 3000)
        cfg = {"mid": core.sched_cfg(T_e=400, M_e=500, refine_epochs=()),
               "diff": core.sched_cfg(T_e=1600, M_e=2000, refine_epochs=())}.get(
            name, core.sched_cfg(T_e=2600, M_e=3000, refine_epochs=(1000, 2000)))
        # large-growth: a growth round of 256 kernels from the top-1% residual
        # points every 40 steps as well (1k -> 16k within the first 2600 steps)
        add_every = 40 if name == "large-growth" else 0
        def progress(i, row):
            if (i + 1) % 250 == 0:
                r = row[0]
                log(f"{name}: step {i + 1}, L2 {r['L2']:.4g}, kernels {r['m']}, l1 {r['l1']}, "
                    f"b_f {r['b_f']}, levels {fit.next_level[0]}")
        _, lg = fit.fit_schedule(steps, cfg, top_frac=0.01, k_new=256, on_step=progress, add_every=add_every,
                                 **tau)
        n_add = sum(r[0]["n_added"] for r in lg)
        n_prune = sum(r[0]["n_pruned"] for r in lg)
    wall = time.perf_counter() - t0
    st = fit.stats()[0]
    m_final = int(fit.m_dev.item())
    finest = len(prob.levels) - 1
    t1 = time.perf_counter()
    hd, cd, cs = fit.surface_metrics(0, finest, n_samples=100000, seed=1)
    ms_eval = 1e3 * (time.perf_counter() - t1)
    finite = math.isfinite(hd)
    out = {"config": name, "steps": steps, "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
           "final_L2": st.L2, "n_idall": st.n_idall, "kernels_initial": prob.m, "kernels_final": m_final,
           "kernels_added": n_add, "kernels_pruned": n_prune, "overflow": bool(st.flags),
           "pairs_last_step": st.P_fwd + st.P_bwd, "HD": hd if finite else None, "CD": cd if finite else None,
           "CS": cs, "surface": "ok" if finite else "fitted field has no zero crossing",
           "metrics_ms": ms_eval, "levels": [lv.n for lv in prob.levels]}
    if name != "tiny":
        # the same step without the control and its one host wait per step:
        # 100 plain steps from the final state, after the metrics
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(100):
            fit.step(mode=L.MODE_DYNAMIC, lr=1e-5, **tau)
        torch.cuda.synchronize()
        out["ms_per_step_plain_final_state"] = 1e3 * (time.perf_counter() - t1) / 100
    if name == "diff":
        out["autograd"] = autograd_steps(fit, 20)
    log(f"{name}: {steps} steps in {wall:.2f} s ({out['ms_per_step']:.3f} ms/step), L2 {st.L2:.4g}, kernels "
        f"{prob.m} -> {m_final}, HD {hd:.4g} CD {cd:.4g} CS {cs:.4f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes of the CPU baseline (0: every host CPU, at most 16)")
    ap.add_argument("--graph", action="store_true", help="also time HIP-graph replays of the step")
    ap.add_argument("--no-batching", action="store_true", help="leave out the 64-shape batched-vs-plain comparison")
    ap.add_argument("--batching-steps", type=int, default=5)
    ap.add_argument("--workload-cache", default="",
                    help="npz file of the generated timing workload: read if present, else written")
    ap.add_argument("--gen-only", action="store_true", help="generate (and cache) the workload, then exit")
    ap.add_argument("--no-e2e", action="store_true",
                    help="leave the 128^3 scheduled fit (500 steps) out of the default line")
    ap.add_argument("--e2e", default="",
                    help="run one configuration end to end (tiny, mid, large, diff, batching) and print its JSON")
    ap.add_argument("--variant", type=int, default=-1,
                    help="launch variant of the tile kernels (erbf_set_variant); default: the library's")
    ap.add_argument("--slot-chunk", type=int, default=-1,
                    help="XCD runs of tiles of the grid launches (erbf_set_launch); default: the library's")
    ap.add_argument("--bucket-rank", type=int, default=-1,
                    help="1: ranked tile lists, 0: radix-sorted (erbf_set_launch); default: the library's")
    ap.add_argument("--fwd-chunk", type=int, default=-1,
                    help="kernel records staged per forward chunk: 64, 128 or 256; default: the library's")
    ap.add_argument("--bwd-waves", type=int, default=-1,
                    help="waves per backward tile workgroup: 2, 4 or 8; default: the library's")
    ap.add_argument("--tile-order", type=int, default=-1,
                    help="1: tile kernels take the longest lists first, 0: slot order (default: the library's)")
    ap.add_argument("--init", action="store_true", help="add the inscribed-sphere initialisation timing")
    ap.add_argument("--minibatch", action="store_true", help="add the mini-batch step timing (B_s = 10000)")
    ap.add_argument("--octree", action="store_true", help="add the step on octree layers")
    ap.add_argument("--samples", action="store_true", help="add the step with 40000 surface samples")
    ap.add_argument("--surface", action="store_true", help="add the surface evaluation (HD / CD / CS) timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help=f"copy {COPY_CAL_BYTES} bytes device-to-device before the warm-up (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU (the fit is not sharded across GPUs); --gpus must be 1"}))
        sys.exit(2)

    if args.e2e:
        print(json.dumps(e2e_bench(args.e2e)), flush=True)
        return
    import synth
    from synth import sdf as synth_sdf

    # Everything that forks runs here, before anything touches the GPU, and
    # not at all under a profiler: the SDF sampling pool, and the fork server
    # of the oracle's workers (the CPU baseline).
    profiled = under_profiler()
    if profiled:
        synth_sdf.DEFAULT_WORKERS = 1
        if not args.no_cpu_baseline:
            log("under a profiler: no CPU baseline (its workers would fork)")
            args.no_cpu_baseline = True
        # the profile covers the benchmark step alone
        args.no_e2e = True
    t_setup = time.perf_counter()
    if args.workload_cache and os.path.exists(args.workload_cache):
        prob = synth.load_problem(args.workload_cache)
        log(f"workload read from {args.workload_cache}")
    else:
        prob = synth.make_large_snapshot()
        log(f"workload generated in {time.perf_counter() - t_setup:.1f} s")
        if args.workload_cache:
            synth.save_problem(prob, args.workload_cache)
    if args.gen_only:
        return
    bprobs = None
    if not args.no_batching:
        t0 = time.perf_counter()
        bprobs = synth.make_batching()
        log(f"batching workload generated in {time.perf_counter() - t0:.1f} s")
    mid_prob = None
    if not args.no_e2e:
        mid_prob = synth.make_mid()
    n_cpu = args.cpu_workers or max(1, min(16, os.cpu_count() or 1))
    if not profiled:
        # the fork server of the oracle's and the SDF sampler's workers,
        # started while nothing here has touched the GPU
        from oracle import pool
        pool.start_server()

    import torch
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd.fit import Fitter, ShapeInput

    shape = ShapeInput.from_problem(prob)
    t0 = time.perf_counter()
    fit = Fitter([shape], cull_k=prob.cull_k, all_levels=False)
    refine_ms = []
    for _ in prob.levels:
        r0 = time.perf_counter()
        fit.refine(0)
        refine_ms.append(1e3 * (time.perf_counter() - r0))
    torch.cuda.synchronize()
    log(f"device set-up {time.perf_counter() - t0:.1f} s; refine ms {refine_ms}")

    if args.copy_calibration:
        src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=fit.dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: 3 device copies of {COPY_CAL_BYTES} bytes")

    launch = fit.ctx.erbf_get_launch()
    for key, val in (("variant", args.variant), ("slot_chunk", args.slot_chunk),
                     ("bucket_rank", args.bucket_rank), ("fwd_chunk", args.fwd_chunk),
                     ("bwd_waves", args.bwd_waves), ("tile_order", args.tile_order)):
        if val >= 0:
            launch[key] = val
    fit.ctx.erbf_set_launch_dict(launch)
    launch = fit.ctx.erbf_get_launch()
    variant = launch["variant"]
    kw = dict(mode=L.MODE_DYNAMIC, l1_active=True, lr=prob.lr)
    for _ in range(args.warmup):
        fit.step(**kw)
    torch.cuda.synchronize()
    st = fit.stats()[0]
    if st.flags:
        raise SystemExit(f"bucket overflow: need {st.n_bucket_pairs} entries")
    log(f"warm-up done: P_fwd={st.P_fwd} P_bwd={st.P_bwd} n_idall={st.n_idall} L2={st.L2:.4g}")

    fit.ctx.reset_stats()
    fit.ctx.erbf_timing_enable(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fit.step(**kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms, bt_ms, br_ms, ncalls = fit.ctx.erbf_timing_read()
    st = fit.stats()[0]
    K = args.steps
    assert ncalls == K and st.calls == K and st.flags == 0
    P_fwd, P_bwd = st.P_fwd_total, st.P_bwd_total
    ms_per_step = 1e3 * wall / K
    pairs_per_step = (P_fwd + P_bwd) / K
    value = (P_fwd + P_bwd) / wall
    fwd_avg, bt_avg, br_avg = fwd_ms / K, bt_ms / K, br_ms / K
    fused = (variant & L.VARIANT_FUSED) != 0
    if fused:
        # one kernel forms f, the loss and the backward moments of every tile
        # (the reduce kernel only sums per-tile moments)
        fwd_rate = bwd_rate = None
        ach = (FWD_FLOP_PER_PAIR * P_fwd + BWD_FLOP_PER_PAIR * P_bwd) / K / (fwd_avg * 1e-3)
        dom, dom_short, t_dom = "k_step_tiles (forward + loss + backward moments)", "k_step_tiles", fwd_avg
    else:
        fwd_rate = FWD_FLOP_PER_PAIR * P_fwd / K / (fwd_avg * 1e-3)
        # the backward's per-pair arithmetic runs in the tile kernel
        bwd_rate = BWD_FLOP_PER_PAIR * P_bwd / K / (bt_avg * 1e-3)
        if bt_avg >= fwd_avg:
            dom, dom_short, ach, t_dom = "k_bwd_tiles (backward moments)", "k_bwd_tiles", bwd_rate, bt_avg
        else:
            dom, dom_short, ach, t_dom = "k_forward (forward + loss)", "k_forward", fwd_rate, fwd_avg
    # HBM bytes per launch from the committed counter summary, if it was
    # taken on the current kernel source
    from paper_2505_02350_amd.prof_summary import read_traffic
    tb = read_traffic(TRAFFIC_FILE)
    traffic = None
    if tb is not None and dom_short in tb.get("kernels", {}):
        traffic = tb["kernels"][dom_short]["traffic_bytes_per_launch"]
    if fused:
        log(f"timed {K} steps: {ms_per_step:.3f} ms/step; step tiles (forward + backward) {fwd_avg:.3f} ms, "
            f"reduce {br_avg:.3f} ms")
    else:
        log(f"timed {K} steps: {ms_per_step:.3f} ms/step; forward {fwd_avg:.3f} ms, backward tiles "
            f"{bt_avg:.3f} ms, reduce {br_avg:.3f} ms")

    graph_ms = graph10_ms = None
    if args.graph:
        for per in (1, 10):
            fit.capture(steps_per_graph=per, **kw)
            for _ in range(2):
                fit.replay()
            torch.cuda.synchronize()
            reps = max(1, K // per)
            t0 = time.perf_counter()
            for _ in range(reps):
                fit.replay()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / (reps * per)
            if per == 1:
                graph_ms = ms
            else:
                graph10_ms = ms
        log(f"graph replay: {graph_ms:.3f} ms per step (one step per graph), {graph10_ms:.3f} ms (ten per graph)")

    out = {
        "metric": "fwd+bwd ERBF point-kernel pairs/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large_snapshot: smooth union of 12 boxes + 6 capsules + 4 tori on 64^3 + 128^3 + "
                        "256^3 (|S|<0.1) grid levels, 16384 ERBFs, cull 3/min-scale, seed 2",
            "points": int(sum(lv.n ** 3 for lv in prob.levels[:2]) + int(np.count_nonzero(np.abs(prob.levels[2].S) < 0.1))),
            "kernels": prob.m,
            "pairs_per_step": pairs_per_step,
            "P_fwd_per_step": P_fwd / K,
            "P_bwd_per_step": P_bwd / K,
            "mode": "dynamic (eq. 3-21), Adam lr 1e-2",
        },
        "roofline": {
            "bound": "alu",
            "kernel": dom,
            "kernel_ms": t_dom,
            "achieved": ach / 1e12,
            "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": ach / FP32_VECTOR_PEAK,
            "traffic": traffic,
        },
        "kernels_ms": ({"step_tiles": fwd_avg, "backward_reduce": br_avg} if fused else
                       {"forward": fwd_avg, "backward_tiles": bt_avg, "backward_reduce": br_avg,
                        "forward_tflops": fwd_rate / 1e12, "backward_tflops": bwd_rate / 1e12}),
        "launch": launch,
        "fwd_bwd_pairs_per_s": (P_fwd + P_bwd) / ((fwd_ms + bt_ms + br_ms) * 1e-3),
        "bucket_entries": st.n_bucket_pairs,
        "graph_ms_per_step": graph_ms,
        "graph10_ms_per_step": graph10_ms,
        "per_level_refine_ms": refine_ms,
    }
    if bprobs is not None:
        out["batching"] = batching_bench(bprobs, args.batching_steps, 2)
    if mid_prob is not None:
        out["end_to_end"] = e2e_bench("mid", mid_prob)
    if args.init:
        out["init"] = init_bench(with_cpu=not args.no_cpu_baseline)
    if args.minibatch:
        out["minibatch"] = minibatch_bench(max(args.steps, 20), args.warmup)
    if args.octree:
        out["octree"] = variant_bench("octree", args.steps, args.warmup)
    if args.samples:
        out["samples"] = variant_bench("samples", args.steps, args.warmup)
    if args.surface:
        out["surface"] = surface_bench(with_cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(prob, n_cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
