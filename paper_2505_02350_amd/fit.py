"""Host-side driving of optimisation steps through the C ABI.

:class:`Fitter` owns a library context, the device copies of one or more
shapes' inputs, parameters and Adam moments, and runs steps either eagerly or
as a replayed HIP graph.  Targets and band masks are produced on the device
by the library (eq. 3-10 and the band rule); nothing here computes the
method's arithmetic.
"""

import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from . import core


def estimate_pair_cap(level_ns: Sequence[int], s_min: np.ndarray, cull_k: float,
                      slack: float = 1.5) -> int:
    """Upper estimate of tile-list entries: tiles met by each ball's box."""
    r = cull_k / np.exp(np.asarray(s_min, np.float64))
    tot = 0.0
    for n in level_ns:
        tile = 8 * 2.0 / n
        nt = math.ceil(n / 8)
        per = np.minimum(2 * r / tile + 2, nt) ** 3
        tot += per.sum()
    return int(min(tot * slack + 4096, 2 ** 31 - 1))


class ShapeInput:
    """Host inputs of one shape: level resolutions, axes, raw SDFs, bands,
    which levels are octree layers below the previous one, and which are
    surface-sample levels (samples[i]: float32 (K, 3) points, sample_caps[i]
    their index slots; axes/sdfs/bands entries of such a level are None)."""

    def __init__(self, level_ns, axes, sdfs, bands, params, m, cap, octree=None, samples=None, sample_caps=None):
        self.level_ns = list(level_ns)
        self.axes = list(axes)
        self.sdfs = list(sdfs)
        self.bands = list(bands)
        self.octree = list(octree) if octree is not None else [False] * len(self.level_ns)
        self.samples = list(samples) if samples is not None else [None] * len(self.level_ns)
        self.sample_caps = list(sample_caps) if sample_caps is not None else [0] * len(self.level_ns)
        self.params = np.asarray(params, np.float32)
        self.m = int(m)
        self.cap = int(cap)

    @classmethod
    def from_problem(cls, prob):
        return cls([lv.n for lv in prob.levels], [lv.axis for lv in prob.levels],
                   [lv.S for lv in prob.levels], [lv.band for lv in prob.levels], prob.params, prob.m,
                   prob.cap, [lv.octree for lv in prob.levels], [lv.samples for lv in prob.levels],
                   [lv.sample_cap if lv.samples is not None else 0 for lv in prob.levels])

    def s_min(self):
        seg = self.params.reshape(11, self.cap)[:, :self.m]
        return seg[4:7].min(axis=0)


class Fitter:
    """Library context + device state for a set of shapes, one level each
    registered up front (or all levels when ``all_levels``)."""

    def __init__(self, shapes: List[ShapeInput], cull_k: float = 3.0, weight_map: int = 0,
                 pair_cap: Optional[int] = None, all_levels: bool = True, device: int = 0,
                 orientation: int = L.ORIENT_QUATERNION, batch_cap: int = 0):
        self.shapes = shapes
        self.dev = torch.device("cuda", device)
        if pair_cap is None:
            pair_cap = sum(estimate_pair_cap(s.level_ns, s.s_min(), cull_k) for s in shapes)
        self.ctx = core.Context([(s.level_ns, s.cap, s.sample_caps) for s in shapes], pair_cap, cull_k, weight_map,
                                device, orientation, batch_cap)
        self._levels = []
        # eq. 3-10's m: minimum over every level of a shape, computed on the device
        self.m_sdf = torch.zeros(len(shapes), dtype=torch.float32, device=self.dev)
        self.S_dev = []
        for b, s in enumerate(shapes):
            row = []
            first = True
            for li, S in enumerate(s.sdfs):
                if s.samples[li] is not None:   # surface samples: no grid SDF
                    row.append(torch.from_numpy(np.ascontiguousarray(s.samples[li], np.float32)).to(self.dev))
                    continue
                Sd = torch.from_numpy(np.ascontiguousarray(S, np.float32)).to(self.dev)
                core.erbf_sdf_min(Sd, self.m_sdf[b:b + 1], accumulate=not first)
                first = False
                row.append(Sd)
            self.S_dev.append(row)
        m_host = self.m_sdf.cpu().numpy()
        self.next_level = [0] * len(shapes)
        self._bits = [[] for _ in shapes]
        self._m_host = m_host
        if all_levels:
            for b, s in enumerate(shapes):
                for _ in s.level_ns:
                    self.refine(b)
        cap_total = self.ctx.cap_total
        self.p = torch.zeros(11 * cap_total, dtype=torch.float32, device=self.dev)
        pv = self.p.view(11, cap_total)
        for b, s in enumerate(shapes):
            kb = self.ctx.kbase[b]
            pv[:, kb:kb + s.cap] = torch.from_numpy(s.params.reshape(11, s.cap)).to(self.dev)
        self.m_dev = torch.tensor([s.m for s in shapes], dtype=torch.int32, device=self.dev)
        self.m1 = torch.zeros_like(self.p)
        self.m2 = torch.zeros_like(self.p)
        self.step_dev = torch.zeros(len(shapes), dtype=torch.int32, device=self.dev)
        self.grad = torch.zeros_like(self.p)
        self.graph = None

    def refine(self, b: int):
        """Append shape b's next level (targets and band mask made on device)."""
        s = self.shapes[b]
        li = self.next_level[b]
        Sd = self.S_dev[b][li]
        if s.samples[li] is not None:
            self.ctx.erbf_refine_samples(b, Sd)
            self._bits[b].append(None)
            self._levels.append((Sd,))
            self.next_level[b] += 1
            return
        ax = torch.from_numpy(np.ascontiguousarray(s.axes[li], np.float32)).to(self.dev)
        t = core.erbf_targets_from_sdf(Sd, float(self._m_host[b]))
        if s.octree[li]:
            bits = core.erbf_octree_bits(self.S_dev[b][li - 1], s.level_ns[li - 1], self._bits[b][li - 1])
        else:
            bits = core.erbf_band_bits(Sd, s.bands[li]) if s.bands[li] is not None else None
        self._bits[b].append(bits)
        self._levels.append((ax, t, bits))
        self.ctx.erbf_refine_level(b, ax, t, Sd, bits)
        self.next_level[b] += 1

    def step(self, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None, l1_active=False, lr=1e-3, lr_dev=None,
             tau1=0.9, tau2=1.1, tau_m=0.02, stream=None):
        self.ctx.erbf_train_step(self.p, self.m_dev, self.grad, self.m1, self.m2, self.step_dev, mode=mode, lam=lam,
                                 lambda_dev=lambda_dev, l1_active=l1_active, tau1=tau1, tau2=tau2, tau_m=tau_m,
                                 lr=lr, lr_dev=lr_dev, stream=stream)

    def capture(self, steps_per_graph: int = 1, **kw):
        """Capture `steps_per_graph` consecutive steps into one HIP graph
        (replay with :meth:`replay`)."""
        s = torch.cuda.Stream(device=self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            self.step(stream=s, **kw)   # warm-up outside the graph
        torch.cuda.current_stream(self.dev).wait_stream(s)
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for _ in range(int(steps_per_graph)):
                self.step(stream=s, **kw)
        self.graph = g
        self.graph_steps = int(steps_per_graph)
        return g

    def replay(self):
        self.graph.replay()

    def stats(self):
        return self.ctx.stats()

    def fit_schedule(self, steps: int, cfg=None, tau1: float = 0.9, tau2: float = 1.1, tau_m: float = 0.02,
                     top_frac: float = 0.01, k_new: int = 256, min_abs_err: float = 0.0, stream=None,
                     on_step=None, add_every: int = 0, state=None, lagged: bool = True):
        """Algorithm 3 on every shape for `steps` full-batch steps.

        Each step: loss and gradient with eq. 3-21 gated by the device control
        state and Adam with the state's learning rate (one erbf_train_step),
        then the control itself (pruning by eq. 3-27 happens there, on the
        device).  When the control asks for new kernels (eq. add_activate) the
        shape is seeded from the step's residual (Algorithm 2) before the next
        step; when it asks for the next grid level, the level is appended
        (eq. 3-16).  The host reads one copy of the requests, counts and
        statistics per step.  With ``lagged`` it does so while the next step
        already runs: the control's hold word makes a step that follows a
        request change nothing, and after the requests are handled that step
        is taken again, so the trajectory is the one of waiting for every
        step (``lagged=False``).  Returns the control state and a per-step
        log of (L2, m, b_f, l1_active, n_added, n_pruned) per shape;
        ``on_step(i, row)``, when given, is called with each step's log row.
        ``add_every`` > 0 also seeds every shape after each add_every-th step
        (a fixed growth round, next to the control's own requests) until the
        final phase.  ``state``: a control state to continue from (one made
        for this context and ``cfg``, e.g. restored by :meth:`load`); by
        default a fresh one.
        """
        cfg = cfg or core.sched_cfg()
        if state is None:
            st = core.SchedState(self.ctx, cfg)
            self.ctx.erbf_sched_init(cfg, st, stream=stream)
        else:
            st = state
        n = len(self.shapes)
        rows = {f: i for i, f in enumerate(core.SchedState.FLAG_ROWS)}
        # two slots: a step's G and the copies of its control flags and
        # statistics go to the slot it was given
        Gs = [torch.zeros(self.ctx.n_points, dtype=torch.float32, device=self.dev) for _ in range(2)]
        snaps = [torch.empty(tuple(st.flags.shape), dtype=torch.int32, pin_memory=True) for _ in range(2)]
        stats_hs = [torch.empty_like(self.ctx.stats_buf, device="cpu").pin_memory() for _ in range(2)]
        done = [torch.cuda.Event() for _ in range(2)]
        s_obj = stream if stream is not None else torch.cuda.current_stream(self.dev)
        m_host = self.m_dev.cpu().tolist()
        log = []

        def enqueue(k):
            with torch.cuda.stream(s_obj):
                self.ctx.erbf_train_step(self.p, self.m_dev, self.grad, self.m1, self.m2, self.step_dev,
                                         mode=L.MODE_DYNAMIC, l1_active_dev=st.l1_active, tau1=tau1, tau2=tau2,
                                         tau_m=tau_m, lr_dev=st.lr, G_out=Gs[k], hold_dev=st.hold if lagged else None,
                                         stream=stream)
                self.ctx.erbf_sched_step(self.p, self.m_dev, cfg, st, self.m1, self.m2, hold=lagged, stream=stream)
                snaps[k].copy_(st.flags, non_blocking=True)
                stats_hs[k].copy_(self.ctx.stats_buf, non_blocking=True)
                done[k].record(s_obj)

        def growth_after(i):
            return add_every > 0 and (i + 1) % add_every == 0

        k = 0
        if steps > 0:
            enqueue(k)
        while len(log) < steps:
            i = len(log)
            # the next step goes in before this one is read, unless the host
            # will change the state in between anyway (a growth round)
            ahead = lagged and i + 1 < steps and not growth_after(i)
            if ahead:
                enqueue(1 - k)
            done[k].synchronize()
            stats = core.parse_stats(stats_hs[k], n)
            for b in range(n):
                if stats[b].flags & L.FLAG_BUCKET_OVERFLOW:
                    raise RuntimeError(f"tile lists overflowed at step {i} (shape {b}): "
                                       f"{stats[b].n_bucket_pairs} entries needed; build the Fitter with a "
                                       f"larger pair_cap")
            add, ref, l1, b_f, n_pr, fin = (snaps[k][rows[f]].tolist() for f in
                                            ("add_request", "refine_request", "l1_active", "b_f", "n_pruned",
                                             "final_phase"))
            # the device's own record of whether it held the following step
            requested = lagged and int(snaps[k][rows["hold"]][0]) != 0
            if requested and ahead:
                # the step enqueued ahead was held: it changed nothing
                done[1 - k].synchronize()
            # the live counts follow from the pruning counts and the seeding
            m_now = [m_host[b] - n_pr[b] for b in range(n)]
            grow = growth_after(i)
            row = []
            for b, s in enumerate(self.shapes):
                n_added = 0
                room = s.cap - m_now[b]
                if (add[b] or (grow and not fin[b])) and room > 0 and stats[b].n_idall > 0:
                    n_added = self.ctx.erbf_seed_from_error(self.p, self.m_dev, b, Gs[k], 0.5, stats[b].n_idall,
                                                            top_frac=top_frac, k_new=min(k_new, room),
                                                            min_abs_err=min_abs_err, m1=self.m1, m2=self.m2,
                                                            stream=stream)
                if ref[b] and self.next_level[b] < len(s.level_ns):
                    self.refine(b)
                m_host[b] = m_now[b] + n_added
                row.append(dict(L2=stats[b].L2, m=m_host[b], l1=bool(l1[b]), b_f=int(b_f[b]),
                                n_added=n_added, n_pruned=int(n_pr[b])))
            log.append(row)
            if on_step is not None:
                on_step(i, row)
            if requested:
                with torch.cuda.stream(s_obj):
                    st.hold.zero_()
            k = 1 - k
            if len(log) < steps and (requested or not ahead):
                # no step in flight that counts: enqueue the next one
                enqueue(k)
        return st, log

    # ---- checkpoint / resume --------------------------------------------------
    def save(self, path: str, sched: "core.SchedState" = None):
        """Write the fit's state to an ``.npz`` file (no pickles): parameters,
        Adam moments and step counters, live counts, registered levels per
        shape and, when given, the training control's state.  Resuming with
        :meth:`load` into a Fitter built from the same shapes continues the
        fit bit for bit."""
        torch.cuda.synchronize(self.dev)
        arrs = {"p": self.p.cpu().numpy(), "m1": self.m1.cpu().numpy(), "m2": self.m2.cpu().numpy(),
                "step": self.step_dev.cpu().numpy(), "m": self.m_dev.cpu().numpy(),
                "levels": np.asarray(self.next_level, np.int32)}
        if sched is not None:
            for f, _ in L.SchedState._fields_:
                arrs["sched_" + f] = getattr(sched, f).cpu().numpy()
        np.savez(path, **arrs)

    def load(self, path: str, sched: "core.SchedState" = None):
        """Restore a state written by :meth:`save` (levels not yet registered
        here are appended first; the shapes must be the ones it was saved
        from)."""
        z = np.load(path, allow_pickle=False)
        levels = z["levels"].tolist()
        if len(levels) != len(self.shapes):
            raise ValueError("checkpoint holds a different number of shapes")
        for b, want in enumerate(levels):
            if self.next_level[b] > want:
                raise ValueError("checkpoint has fewer registered levels than this fitter")
            while self.next_level[b] < want:
                self.refine(b)
        for name, t in (("p", self.p), ("m1", self.m1), ("m2", self.m2), ("step", self.step_dev),
                        ("m", self.m_dev)):
            a = z[name]
            if a.shape != tuple(t.shape):
                raise ValueError(f"checkpoint field {name} has shape {a.shape}, expected {tuple(t.shape)}")
            t.copy_(torch.from_numpy(a))
        if sched is not None:
            for f, _ in L.SchedState._fields_:
                if "sched_" + f in z.files:
                    getattr(sched, f).copy_(torch.from_numpy(z["sched_" + f]))
                elif f != "hold":
                    raise ValueError(f"checkpoint has no control field {f}")
        torch.cuda.synchronize(self.dev)

    def init_inscribed(self, b: int = 0, gamma: float = 1e-3, max_centres: int = 0, stream=None):
        """Replace shape b's kernels by the inscribed-sphere initialisation
        (Algorithm 1, eq. 3-12) over its registered levels (with its surface
        samples, if registered, giving the depth); restarts its Adam state.
        Returns (centres, candidates left uncovered)."""
        nc, left = self.ctx.erbf_init_inscribed(self.p, self.m_dev, b, gamma=gamma, max_centres=max_centres,
                                                m1=self.m1, m2=self.m2, stream=stream)
        self.step_dev[b:b + 1].zero_()
        return nc, left

    def surface_metrics(self, b: int, li: int, n_samples: int = 100000, seed: int = 0, stream=None):
        """Section 4's HD / CD / CS between the zero set of grid level li's
        signed distance and that of the fitted field on the same grid (the
        network's output taken back through eq. 3-10), each sampled at
        n_samples area-uniform points from seeded uniforms."""
        s = self.shapes[b]
        if s.samples[li] is not None:
            raise ValueError("level li must be a grid level")
        n = s.level_ns[li]
        f = self.ctx.erbf_eval(self.p, self.m_dev, stream=stream)
        base = self.ctx.pt_base[b][li]
        Sr = core.erbf_sdf_from_targets(f[base:base + n ** 3], float(self._m_host[b]), stream=stream)
        ax = torch.from_numpy(np.ascontiguousarray(s.axes[li], np.float32)).to(self.dev)
        rng = np.random.default_rng(seed)
        out = []
        for field in (self.S_dev[b][li], Sr):
            tris = core.erbf_surface_extract(field, n, ax, 0.0, stream=stream)
            if tris.shape[0] == 0:
                return float("inf"), float("inf"), 0.0
            u = torch.from_numpy(rng.random((n_samples, 3)).astype(np.float32)).to(self.dev)
            pts, nrm, _ = core.erbf_surface_sample(tris, u, stream=stream)
            out.append((pts, nrm))
        return core.erbf_surface_metrics(out[0][0], out[0][1], out[1][0], out[1][1], stream=stream)

    def training_points(self, b: int) -> np.ndarray:
        """Indices (into the context's per-point arrays) of shape b's training
        points: every point of its registered levels inside the level's band."""
        s = self.shapes[b]
        out = []
        for li in range(self.next_level[b]):
            if s.samples[li] is not None:
                out.append(self.ctx.pt_base[b][li] + np.arange(len(s.samples[li])))
                continue
            S = np.asarray(s.sdfs[li], np.float32).reshape(-1)
            if self._bits[b][li] is not None:
                words = self._bits[b][li].cpu().numpy().view(np.uint32)
                keep = np.unpackbits(words.view(np.uint8), bitorder="little")[:S.size].astype(bool)
            else:
                keep = np.ones(S.size, bool)
            out.append(self.ctx.pt_base[b][li] + np.nonzero(keep)[0])
        return np.concatenate(out).astype(np.int64)

    def fit_minibatch(self, epochs: int, batch_size: int, seed: int = 0, mode=L.MODE_FIXED, lam=0.0,
                      lr=1e-3, tau1=0.9, tau2=1.1, tau_m=0.02, l1_active=False, stream=None):
        """Mini-batch epochs (Algorithm 3's inner loop): each epoch shuffles the
        training points of every shape (seeded permutation, an input) and
        takes one loss + gradient + Adam step per batch of `batch_size`
        points.  Returns the per-batch L2 of shape 0."""
        if batch_size > self.ctx.batch_cap:
            raise ValueError("batch_size exceeds the context's batch_cap")
        pts = np.concatenate([self.training_points(b) for b in range(len(self.shapes))])
        log = []
        for ep in range(epochs):
            perm = np.random.default_rng([seed, ep]).permutation(pts.size)
            order = torch.from_numpy(pts[perm]).to(self.dev)
            for i in range(0, pts.size, batch_size):
                idx = order[i:i + batch_size]
                self.ctx.erbf_loss_grad_minibatch(self.p, self.m_dev, idx, mode=mode, lam=lam, l1_active=l1_active,
                                              tau1=tau1, tau2=tau2, tau_m=tau_m, grad_out=self.grad, stream=stream)
                self.ctx.erbf_adam_step(self.p, self.m_dev, self.grad, self.m1, self.m2, self.step_dev, lr=lr,
                                        stream=stream)
                log.append(self.ctx.stats()[0].L2)
        return log


def jsonl_logger(path: str):
    """An ``on_step`` callback for :meth:`Fitter.fit_schedule` that appends
    each step's per-shape row (L2, kernel count, b_f, L1 flag, kernels added
    and pruned) to a JSON-lines file."""
    import json

    def on_step(i, row):
        with open(path, "a") as fh:
            fh.write(json.dumps({"step": i, "shapes": row}) + "\n")
    return on_step
