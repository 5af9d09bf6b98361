"""Shared set-up of GPU parity tests: build a library context and the oracle's
view of the same synthetic problem.

Inputs flow one way: synth -> (oracle, GPU).  Targets are computed by the
oracle (eq. 3-10, float64, stored float32) and uploaded; nothing the GPU
computes is handed to the oracle.
"""

import json
import math
import os

import numpy as np

import oracle as O

TAU1 = float(np.float32(0.9))
TAU2 = float(np.float32(1.1))
TAU_M = float(np.float32(0.02))

# measured errors of the parity tests go here (a folder of the caller's
# choice, else parity_records/ at the repository root)
RESULTS = os.environ.get("ERBF_PARITY_DIR") or os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "parity_records")


def record(name, **vals):
    """Write the measured errors of a parity test (and print them)."""
    os.makedirs(RESULTS, exist_ok=True)
    with open(os.path.join(RESULTS, f"{name}.json"), "w") as fh:
        json.dump(vals, fh, indent=1, default=float)
    print(name, json.dumps(vals, default=float), flush=True)


def oracle_levels(prob, with_targets=True):
    S_all = [lv.S for lv in prob.levels if lv.samples is None]
    m = O.sdf_min(S_all)
    out, t32 = [], []
    for li, lv in enumerate(prob.levels):
        if lv.samples is not None:
            out.append(O.make_samples(lv.samples, lv.sample_cap))
            t32.append(None)
            continue
        t = O.targets_from_sdf(lv.S, m).astype(np.float32) if with_targets else None
        t32.append(t)
        if lv.octree:
            par = prob.levels[li - 1]
            act = O.octree_mask(par.S, par.n, out[-1].active)
        else:
            act = lv.active_mask()
        out.append(O.make_level(lv.n, lv.axis, active=act, t=t, S=lv.S))
    return out, t32, m


def pair_cap_estimate(prob, slack=2.0):
    """Generous bound on tile-list entries: tiles touched by each ball's box."""
    seg = prob.params.reshape(11, prob.cap)[:, :prob.m]
    smin = seg[4:7].min(axis=0).astype(np.float64)
    r = prob.cull_k / np.exp(smin)
    tot = 0
    for lv in prob.levels:
        tile = 8 * 2.0 / lv.n
        per = (np.minimum(2 * r / tile + 2, math.ceil(lv.n / 8))) ** 3
        tot += per.sum()
    return int(tot * slack) + 4096


class GpuProblem:
    """A one-shape library context holding `prob`'s levels and parameters."""

    def __init__(self, prob, targets, pair_cap=None, weight_map=None, n_levels=None, batch_cap=0):
        import torch
        from paper_2505_02350_amd import core
        self.torch = torch
        self.prob = prob
        nl = len(prob.levels) if n_levels is None else n_levels
        wm = prob.weight_map if weight_map is None else weight_map
        samp = [lv.sample_cap if lv.samples is not None else 0 for lv in prob.levels[:nl]]
        self.ctx = core.Context([([lv.n for lv in prob.levels[:nl]], prob.cap, samp)],
                                pair_cap or pair_cap_estimate(prob), prob.cull_k, wm,
                                orientation=prob.orientation, batch_cap=batch_cap)
        dev = self.ctx.device
        self.axes, self.tgts, self.sdfs, self.bits = [], [], [], []
        for li, lv in enumerate(prob.levels[:nl]):
            if lv.samples is not None:
                xyz = torch.from_numpy(np.ascontiguousarray(lv.samples, np.float32)).to(dev)
                for lst, v in ((self.axes, None), (self.tgts, None), (self.sdfs, None), (self.bits, None)):
                    lst.append(v)
                self.samples = xyz
                self.ctx.erbf_refine_samples(0, xyz)
                continue
            ax = torch.from_numpy(np.asarray(lv.axis, np.float32)).to(dev)
            S = torch.from_numpy(np.asarray(lv.S, np.float32)).to(dev)
            t = None if targets is None or targets[li] is None else torch.from_numpy(targets[li]).to(dev)
            if lv.octree:
                bits = core.erbf_octree_bits(self.sdfs[li - 1], prob.levels[li - 1].n, self.bits[li - 1])
            else:
                bits = core.erbf_band_bits(S, lv.band) if lv.band is not None else None
            self.axes.append(ax)
            self.tgts.append(t)
            self.sdfs.append(S)
            self.bits.append(bits)
            self.ctx.erbf_refine_level(0, ax, t, S, bits)
        self.p = torch.from_numpy(np.asarray(prob.params, np.float32)).to(dev)
        self.m_dev = torch.tensor([prob.m], dtype=torch.int32, device=dev)
        torch.cuda.synchronize()

    def split_points(self, flat):
        """Per-level numpy arrays from a per-point device array."""
        a = flat.detach().cpu().numpy()
        out = []
        for li, n in enumerate(self.ctx.level_ns[0][:self.ctx.n_active[0]]):
            b = self.ctx.pt_base[0][li]
            k = self.ctx.level_samples[0][li]
            out.append(a[b:b + (k if k > 0 else n ** 3)])
        return out

    def grads_np(self, g):
        a = g.detach().cpu().numpy().astype(np.float64).reshape(11, self.prob.cap)[:, :self.prob.m]
        return {"w": a[0], "c": a[1:4].T, "s": a[4:7].T, "q": a[7:11].T}


def rel_inf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def oracle_grads_dict(gr):
    return {"w": gr.w, "c": gr.c, "s": gr.s, "q": gr.q}


def fd_check(prob, lv, u3, kk, pp, grad, h=1e-6):
    """Check gradients of sum_i u_i f_i on grid level `lv` (u3: the upstream
    as an (n, n, n) array) against FP64 central differences (step h), for the
    (kernel, parameter) pairs (kk[i], pp[i]); parameter index in the packed
    order w, cx, cy, cz, sx, sy, sz, q0..q3.  grad: (m, 11) gradients to check.

    Only kernel j's term moves with its parameters, so each quotient is taken
    on that kernel's own field over its index box with the cull radius doubled
    (oracle.kernel_field), away from the cull boundary.  The checked gradient
    sums the culled terms only: the terms between r and 2 r are the truncation
    allowance, bounded as in the oracle's pins (every dropped pair has
    |D R Delta| >= k_cull), per kernel from the sum of |u| over that shell.
    Returns, per group, the largest (|g - fd| - allowance) / (the group's
    largest |fd|); per group, the largest |g - (fd - shell)| / (that scale),
    shell the oracle's analytic gradient of the terms between r and 2 r (the
    allowance's exact value); and the largest allowance relative to |fd|."""
    import dataclasses
    from oracle import erbf as OE
    P = np.asarray(prob.params, np.float64).reshape(11, prob.cap)
    K = OE.kernels_from_packed(prob.params, prob.m, prob.cap, prob.cull_k, prob.weight_map, prob.orientation)
    k2 = prob.cull_k ** 2
    ek = math.exp(-k2)
    fd, gv, allow, group, shells = [], [], [], [], []
    shell_of = {}
    for j, par in zip(kk, pp):
        def obj(delta):
            Q = P[:, j].copy()
            Q[par] += delta
            Kj = OE.make_kernels(Q[0:1], Q[None, 1:4], Q[None, 4:7], Q[None, 7:11], prob.cull_k, prob.weight_map,
                                 prob.orientation)
            (z0, z1, y0, y1, x0, x1), v = OE.kernel_field(lv, Kj, 0, radius_scale=2.0)
            return float(np.sum(u3[z0:z1, y0:y1, x0:x1] * v))
        fd.append((obj(h) - obj(-h)) / (2 * h))
        gv.append(float(grad[j, par]))
        Kj = OE.subset(K, [j])
        (z0, z1, y0, y1, x0, x1), dx, dy, dz = OE._kernel_box(lv, Kj, 0, 4.0 * Kj.r2[0])
        d2 = dx * dx + dy * dy + dz * dz
        shell = float(np.sum(np.abs(u3[z0:z1, y0:y1, x0:x1]) * ((d2 >= Kj.r2[0]) & (d2 < 4.0 * Kj.r2[0]))))
        a, dmax, dmin = abs(Kj.a[0]), Kj.d[0].max(), Kj.d[0].min()
        if par == 0:
            b = ek * shell * Kj.dadw[0]
        elif par < 4:
            b = 2 * a * dmax * prob.cull_k * ek * shell
        elif par < 7:
            b = 2 * a * k2 * ek * shell
        else:
            J = OE.quat_rot_jacobian(Kj.qhat[0:1])[0].reshape(4, 9)
            b = np.linalg.norm(J, 2) * 2 * a * (dmax / dmin) * k2 * ek * shell / Kj.qn[0]
        allow.append(b)
        group.append(0 if par == 0 else (1 if par < 4 else (2 if par < 7 else 3)))
        if j not in shell_of:
            ge = OE.backward([lv], dataclasses.replace(Kj, r2=4.0 * Kj.r2), [u3.reshape(-1)])
            gc = OE.backward([lv], Kj, [u3.reshape(-1)])
            shell_of[j] = (np.concatenate([ge.w, ge.c[0], ge.s[0], ge.q[0]]) -
                           np.concatenate([gc.w, gc.c[0], gc.s[0], gc.q[0]]))
        shells.append(float(shell_of[j][par]))
    fd, gv, allow, group, shells = map(np.asarray, (fd, gv, allow, group, shells))
    worst, exact = {}, {}
    for gi, name in enumerate(("w", "c", "s", "q")):
        sel = group == gi
        if sel.any():
            scale = np.abs(fd[sel]).max()
            worst[name] = float(((np.abs(gv[sel] - fd[sel]) - allow[sel]) / scale).max())
            exact[name] = float((np.abs(gv[sel] - (fd[sel] - shells[sel])) / scale).max())
    return worst, exact, float((allow / np.maximum(np.abs(fd), 1e-30)).max())
