"""Thin Python surface over the C ABI (``include/erbf.h``).

Names follow the C calls.  Torch supplies device memory and the stream;
this module only marshals pointers and sizes.
"""

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


@dataclass
class StatsView:
    L2: float
    L1: float
    loss: float
    alpha: float
    beta: float
    n_idall: int
    P_fwd: int
    P_bwd: int
    n_bucket_pairs: int
    max_abs_E: float
    m: int
    flags: int
    P_fwd_total: int
    P_bwd_total: int
    calls: int


def parse_stats(buf: torch.Tensor, n_shapes: int) -> List[StatsView]:
    raw = bytes(buf.cpu().numpy().tobytes())
    out = []
    for b in range(n_shapes):
        s = L.Stats.from_buffer_copy(raw[b * L.STATS_BYTES:(b + 1) * L.STATS_BYTES])
        out.append(StatsView(s.L2, s.L1, s.loss, s.alpha, s.beta, s.n_idall, s.P_fwd, s.P_bwd,
                             s.n_bucket_pairs, s.max_abs_E, s.m, s.flags, s.P_fwd_total, s.P_bwd_total,
                             s.calls))
    return out


class Context:
    """One library context: shapes, their grid levels and the workspace."""

    def __init__(self, shapes: Sequence, pair_cap: int, cull_k: float = 3.0,
                 weight_map: int = L.WEIGHT_SIGNED_SQUARE, device: int = 0,
                 orientation: int = L.ORIENT_QUATERNION, batch_cap: int = 0):
        """shapes: sequence of (level_ns, m_cap) or (level_ns, m_cap,
        level_samples): level_samples[i] > 0 makes level i a surface-sample
        level of that capacity, binned on a grid of level_ns[i] cells."""
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        descs = (L.ShapeDesc * len(shapes))()
        self.level_ns = []
        self.level_samples = []
        self.m_caps = []
        for b, sh in enumerate(shapes):
            ns, mcap = [int(n) for n in sh[0]], int(sh[1])
            samp = [int(v) for v in sh[2]] if len(sh) > 2 and sh[2] is not None else [0] * len(ns)
            descs[b].n_levels = len(ns)
            for i, n in enumerate(ns):
                descs[b].level_n[i] = n
                descs[b].level_samples[i] = samp[i]
            descs[b].m_cap = mcap
            self.level_ns.append(ns)
            self.level_samples.append(samp)
            self.m_caps.append(mcap)
        self._descs = descs
        cfg = L.Config(len(shapes), descs, int(pair_cap), float(cull_k), int(weight_map), int(orientation),
                       int(batch_cap))
        self.batch_cap = int(batch_cap)
        self._cfg = cfg
        nbytes = ctypes.c_size_t()
        L.check(self.lib.erbf_workspace_size(ctypes.byref(cfg), ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        h = ctypes.c_void_p()
        L.check(self.lib.erbf_ctx_create(device, ctypes.byref(cfg), aligned, self.ws_bytes, ctypes.byref(h)))
        self.handle = h
        cap = ctypes.c_int32()
        npts = ctypes.c_int64()
        L.check(self.lib.erbf_ctx_info(h, ctypes.byref(cap), ctypes.byref(npts), None))
        self.cap_total = cap.value
        self.n_points = npts.value
        self.n_shapes = len(shapes)
        self.kbase = [sum(self.m_caps[:b]) for b in range(self.n_shapes)]
        # per-point offsets (shape-major over declared levels)
        self.pt_base = []
        off = 0
        for ns, samp in zip(self.level_ns, self.level_samples):
            row = []
            for n, k in zip(ns, samp):
                row.append(off)
                off += k if k > 0 else n ** 3
            self.pt_base.append(row)
        self.n_active = [0] * self.n_shapes
        self._keep = []   # device arrays the context points into
        self.stats_buf = torch.zeros(self.n_shapes * L.STATS_BYTES, dtype=torch.uint8, device=self.device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.erbf_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- levels -------------------------------------------------------------
    def erbf_refine_level(self, shape: int, axis: torch.Tensor, target: torch.Tensor = None,
                          sdf: torch.Tensor = None, active_bits: torch.Tensor = None, stream=None):
        n = self.level_ns[shape][self.n_active[shape]]
        for t, name in ((axis, "axis"), (target, "target"), (sdf, "sdf")):
            if t is not None and t.dtype != torch.float32:
                raise ValueError(f"{name} must be float32")
        if active_bits is not None and active_bits.dtype != torch.int32:
            raise ValueError("active_bits must be int32 words")
        lvl = L.Level(n, _ptr(axis), _ptr(target), _ptr(sdf), _ptr(active_bits), None, 0)
        self._keep.append((axis, target, sdf, active_bits))
        L.check(self.lib.erbf_refine_level(self.handle, shape, ctypes.byref(lvl), _stream(stream)))
        self.n_active[shape] += 1

    def erbf_refine_samples(self, shape: int, xyz: torch.Tensor, stream=None):
        """Register shape's next level, a surface-sample level: xyz float32
        [K, 3] device coordinates in [-1, 1] (label 1)."""
        li = self.n_active[shape]
        n = self.level_ns[shape][li]
        if self.level_samples[shape][li] <= 0:
            raise ValueError("the next declared level is not a sample level")
        if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
            raise ValueError("xyz must be a contiguous float32 [K, 3] tensor")
        lvl = L.Level(n, None, None, None, None, _ptr(xyz), int(xyz.shape[0]))
        self._keep.append((xyz,))
        L.check(self.lib.erbf_refine_level(self.handle, shape, ctypes.byref(lvl), _stream(stream)))
        self.n_active[shape] += 1

    # ---- params ---------------------------------------------------------------
    def new_params(self):
        p = torch.zeros(11 * self.cap_total, dtype=torch.float32, device=self.device)
        m = torch.zeros(self.n_shapes, dtype=torch.int32, device=self.device)
        return p, m

    def _params(self, p: torch.Tensor, m_dev: torch.Tensor):
        if p.dtype != torch.float32 or p.numel() != 11 * self.cap_total:
            raise ValueError("params must be float32 [11 * cap_total]")
        if m_dev.dtype != torch.int32 or m_dev.numel() != self.n_shapes:
            raise ValueError("m_dev must be int32 [n_shapes]")
        return L.Params(_ptr(p), _ptr(m_dev))

    # ---- calls ------------------------------------------------------------------
    def erbf_eval(self, p, m_dev, f_out=None, stats=False, stream=None):
        if f_out is None:
            f_out = torch.zeros(self.n_points, dtype=torch.float32, device=self.device)
        pr = self._params(p, m_dev)
        L.check(self.lib.erbf_eval(self.handle, ctypes.byref(pr), _ptr(f_out),
                                   _ptr(self.stats_buf) if stats else None, _stream(stream)))
        return f_out

    def erbf_loss_grad(self, p, m_dev, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None, l1_active=False,
                       tau1=0.9, tau2=1.1, tau_m=0.02, grad_out=None, f_out=None, G_out=None,
                       l1_active_dev=None, stream=None):
        if grad_out is None:
            grad_out = torch.empty(11 * self.cap_total, dtype=torch.float32, device=self.device)
        pr = self._params(p, m_dev)
        cfg = L.LossCfg(int(mode), float(lam), _ptr(lambda_dev), int(bool(l1_active)), float(tau1),
                        float(tau2), float(tau_m), _ptr(l1_active_dev))
        L.check(self.lib.erbf_loss_grad(self.handle, ctypes.byref(pr), ctypes.byref(cfg), _ptr(grad_out),
                                        _ptr(self.stats_buf), _ptr(f_out), _ptr(G_out), _stream(stream)))
        return grad_out

    def erbf_loss_grad_batched(self, p, m_dev, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None, l1_active=False,
                               tau1=0.9, tau2=1.1, tau_m=0.02, grad_out=None, f_out=None, G_out=None,
                               l1_active_dev=None, stream=None):
        """Loss + gradient of every shape of the context (one launch per stage)."""
        if grad_out is None:
            grad_out = torch.empty(11 * self.cap_total, dtype=torch.float32, device=self.device)
        pr = self._params(p, m_dev)
        cfg = L.LossCfg(int(mode), float(lam), _ptr(lambda_dev), int(bool(l1_active)), float(tau1),
                        float(tau2), float(tau_m), _ptr(l1_active_dev))
        L.check(self.lib.erbf_loss_grad_batched(self.handle, ctypes.byref(pr), ctypes.byref(cfg), _ptr(grad_out),
                                                _ptr(self.stats_buf), _ptr(f_out), _ptr(G_out), _stream(stream)))
        return grad_out

    def erbf_loss_grad_minibatch(self, p, m_dev, pts, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None,
                                 l1_active=False, tau1=0.9, tau2=1.1, tau_m=0.02, grad_out=None, f_out=None,
                                 l1_active_dev=None, stream=None):
        """One mini-batch loss + gradient; pts: int64 device tensor of point indices."""
        if pts.dtype != torch.int64:
            raise ValueError("pts must be int64")
        if grad_out is None:
            grad_out = torch.empty(11 * self.cap_total, dtype=torch.float32, device=self.device)
        pr = self._params(p, m_dev)
        cfg = L.LossCfg(int(mode), float(lam), _ptr(lambda_dev), int(bool(l1_active)), float(tau1),
                        float(tau2), float(tau_m), _ptr(l1_active_dev))
        L.check(self.lib.erbf_loss_grad_minibatch(self.handle, ctypes.byref(pr), ctypes.byref(cfg), _ptr(pts),
                                                  int(pts.numel()), _ptr(grad_out), _ptr(self.stats_buf),
                                                  _ptr(f_out), _stream(stream)))
        return grad_out

    def erbf_vjp(self, p, m_dev, grad_f, grad_out=None, stats=False, stream=None):
        if grad_out is None:
            grad_out = torch.empty(11 * self.cap_total, dtype=torch.float32, device=self.device)
        if grad_f.dtype != torch.float32 or grad_f.numel() != self.n_points:
            raise ValueError("grad_f must be float32 [n_points]")
        pr = self._params(p, m_dev)
        L.check(self.lib.erbf_vjp(self.handle, ctypes.byref(pr), _ptr(grad_f), _ptr(grad_out),
                                  _ptr(self.stats_buf) if stats else None, _stream(stream)))
        return grad_out

    def erbf_adam_step(self, p, m_dev, grad, m1, m2, step_dev, lr=1e-3, lr_dev=None, beta1=0.9,
                       beta2=0.999, eps=1e-8, hold_dev=None, stream=None):
        pr = self._params(p, m_dev)
        cfg = L.AdamCfg(float(lr), _ptr(lr_dev), float(beta1), float(beta2), float(eps), _ptr(hold_dev))
        L.check(self.lib.erbf_adam_step(self.handle, ctypes.byref(pr), _ptr(grad), _ptr(m1), _ptr(m2),
                                        _ptr(step_dev), ctypes.byref(cfg), _stream(stream)))

    def erbf_train_step(self, p, m_dev, grad_out, m1, m2, step_dev, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None,
                        l1_active=False, tau1=0.9, tau2=1.1, tau_m=0.02, l1_active_dev=None, lr=1e-3, lr_dev=None,
                        beta1=0.9, beta2=0.999, eps=1e-8, f_out=None, G_out=None, hold_dev=None, stream=None):
        """Loss, gradient and Adam update in one call (erbf_train_step)."""
        pr = self._params(p, m_dev)
        cfg = L.LossCfg(int(mode), float(lam), _ptr(lambda_dev), int(bool(l1_active)), float(tau1),
                        float(tau2), float(tau_m), _ptr(l1_active_dev))
        acfg = L.AdamCfg(float(lr), _ptr(lr_dev), float(beta1), float(beta2), float(eps), _ptr(hold_dev))
        L.check(self.lib.erbf_train_step(self.handle, ctypes.byref(pr), ctypes.byref(cfg), ctypes.byref(acfg),
                                         _ptr(grad_out), _ptr(m1), _ptr(m2), _ptr(step_dev), _ptr(self.stats_buf),
                                         _ptr(f_out), _ptr(G_out), _stream(stream)))
        return grad_out

    def erbf_seed_from_error(self, p, m_dev, shape, resid, resid_scale, n_idall, top_frac=0.01,
                             k_new=256, r_nms=0.0, eps=1e-7, min_abs_err=0.0, w_rule=0, m1=None, m2=None,
                             stream=None):
        pr = self._params(p, m_dev)
        cfg = L.SeedCfg(float(top_frac), int(k_new), float(r_nms), float(eps), float(min_abs_err), int(w_rule))
        n_added = ctypes.c_int32(0)
        L.check(self.lib.erbf_seed_from_error(self.handle, ctypes.byref(pr), int(shape), _ptr(resid),
                                              float(resid_scale), int(n_idall), ctypes.byref(cfg), _ptr(m1),
                                              _ptr(m2), ctypes.byref(n_added), _stream(stream)))
        return n_added.value

    def erbf_init_inscribed(self, p, m_dev, shape, gamma=1e-3, max_centres=0, m1=None, m2=None, stream=None):
        """Initial kernels of `shape` from inscribed spheres (Algorithm 1,
        eq. 3-12); returns (centres, candidates left uncovered)."""
        pr = self._params(p, m_dev)
        n_c = ctypes.c_int32(0)
        n_left = ctypes.c_int64(0)
        L.check(self.lib.erbf_init_inscribed(self.handle, ctypes.byref(pr), int(shape), float(gamma),
                                             int(max_centres), _ptr(m1), _ptr(m2), ctypes.byref(n_c),
                                             ctypes.byref(n_left), _stream(stream)))
        return n_c.value, n_left.value

    # ---- training control (Algorithm 3) ----------------------------------------
    def erbf_sched_init(self, cfg, state: "SchedState", stream=None):
        L.check(self.lib.erbf_sched_init(self.handle, ctypes.byref(cfg), ctypes.byref(state.c_hold),
                                         _stream(stream)))

    def erbf_sched_step(self, p, m_dev, cfg, state: "SchedState", m1=None, m2=None, hold=False, stream=None):
        """Control after a step; reads this context's stats of the last
        erbf_loss_grad call.  hold: pass the state's hold word (a requesting
        call then holds the calls after it until the word is cleared)."""
        pr = self._params(p, m_dev)
        sc = state.c_hold if hold else state.c
        L.check(self.lib.erbf_sched_step(self.handle, ctypes.byref(pr), ctypes.byref(cfg), ctypes.byref(sc),
                                         _ptr(self.stats_buf), _ptr(m1), _ptr(m2), _stream(stream)))

    def erbf_timing_enable(self, max_calls: int):
        L.check(self.lib.erbf_timing_enable(self.handle, int(max_calls)))

    def erbf_timing_read(self):
        """(forward_ms, backward_tiles_ms, backward_reduce_ms, n_calls), summed."""
        ms = (ctypes.c_double * 3)()
        n = ctypes.c_int32()
        L.check(self.lib.erbf_timing_read(self.handle, ms, ctypes.byref(n)))
        return ms[0], ms[1], ms[2], n.value

    def erbf_set_variant(self, variant: int):
        L.check(self.lib.erbf_set_variant(self.handle, int(variant)))

    def erbf_get_variant(self) -> int:
        v = ctypes.c_int32()
        L.check(self.lib.erbf_get_variant(self.handle, ctypes.byref(v)))
        return v.value

    def erbf_set_launch(self, variant: int, slot_chunk: int, samp_split: int, bucket_rank: int,
                        fwd_chunk: int = 256, bwd_waves: int = 4, tile_order: int = 1):
        c = L.LaunchCfg(int(variant), int(slot_chunk), int(samp_split), int(bucket_rank), int(fwd_chunk),
                        int(bwd_waves), int(tile_order))
        L.check(self.lib.erbf_set_launch(self.handle, ctypes.byref(c)))

    def erbf_get_launch(self):
        """dict of the context's launch choices (erbf_launch_cfg's fields)."""
        c = L.LaunchCfg()
        L.check(self.lib.erbf_get_launch(self.handle, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in L.LaunchCfg._fields_}

    def erbf_set_launch_dict(self, d):
        """Set the launch choices from a dict like erbf_get_launch's."""
        self.erbf_set_launch(**d)

    def erbf_autotune(self, p, m_dev, reps=3, mode=L.MODE_FIXED, lam=0.0, lambda_dev=None, l1_active=False,
                      tau1=0.9, tau2=1.1, tau_m=0.02, stream=None):
        """Choose the fastest launch variant for these parameters; returns
        (variant, per-variant mean milliseconds)."""
        pr = self._params(p, m_dev)
        cfg = L.LossCfg(int(mode), float(lam), _ptr(lambda_dev), int(bool(l1_active)), float(tau1),
                        float(tau2), float(tau_m))
        scratch = torch.empty(11 * self.cap_total, dtype=torch.float32, device=self.device)
        chosen = ctypes.c_int32()
        times = (ctypes.c_float * 8)()
        L.check(self.lib.erbf_autotune(self.handle, ctypes.byref(pr), ctypes.byref(cfg), _ptr(scratch), int(reps),
                                       ctypes.byref(chosen), times, _stream(stream)))
        return chosen.value, list(times)

    def reset_stats(self):
        self.stats_buf.zero_()

    def stats(self) -> List[StatsView]:
        return parse_stats(self.stats_buf, self.n_shapes)


# ---- data preparation ---------------------------------------------------------

def erbf_sdf_min(S: torch.Tensor, out: torch.Tensor, accumulate: bool, stream=None):
    L.check(L.load().erbf_sdf_min(_ptr(S), S.numel(), _ptr(out), int(bool(accumulate)), _stream(stream)))


def erbf_targets_from_sdf(S: torch.Tensor, m: float, t: torch.Tensor = None, stream=None):
    if t is None:
        t = torch.empty_like(S)
    L.check(L.load().erbf_targets_from_sdf(_ptr(S), S.numel(), float(m), _ptr(t), _stream(stream)))
    return t


def erbf_band_bits(S: torch.Tensor, band: float, bits: torch.Tensor = None, stream=None):
    if bits is None:
        bits = torch.empty((S.numel() + 31) // 32, dtype=torch.int32, device=S.device)
    L.check(L.load().erbf_band_bits(_ptr(S), S.numel(), float(band), _ptr(bits), _stream(stream)))
    return bits


def erbf_octree_bits(S_parent: torch.Tensor, n_parent: int, parent_bits: torch.Tensor = None,
                     bits: torch.Tensor = None, stream=None):
    """Active bits of the octree layer (2 n_parent points per axis) below a
    level of n_parent points per axis."""
    nc = 2 * int(n_parent)
    if bits is None:
        bits = torch.empty((nc ** 3 + 31) // 32, dtype=torch.int32, device=S_parent.device)
    L.check(L.load().erbf_octree_bits(_ptr(S_parent), _ptr(parent_bits), int(n_parent), _ptr(bits),
                                      _stream(stream)))
    return bits


# ---- surface evaluation (Section 4) ---------------------------------------------

def erbf_sdf_from_targets(t: torch.Tensor, m: float, out: torch.Tensor = None, stream=None):
    """Signed distance from the normalised field (eq. 3-10 inverted on S >= m)."""
    if out is None:
        out = torch.empty_like(t)
    L.check(L.load().erbf_sdf_from_targets(_ptr(t), t.numel(), float(m), _ptr(out), _stream(stream)))
    return out


def erbf_surface_extract(F: torch.Tensor, n: int, axis: torch.Tensor, iso: float = 0.0, tri_cap: int = None,
                         stream=None):
    """Triangles [T, 3, 3] of the iso-surface of a grid field (marching
    tetrahedra)."""
    lib = L.load()
    nb = ctypes.c_size_t()
    L.check(lib.erbf_surface_scratch_size(int(n), ctypes.byref(nb)))
    scratch = torch.empty(nb.value, dtype=torch.uint8, device=F.device)
    cap = int(tri_cap) if tri_cap is not None else 8 * n * n
    while True:
        tris = torch.empty((max(cap, 1), 3, 3), dtype=torch.float32, device=F.device)
        nt = ctypes.c_int64()
        rc = lib.erbf_surface_extract(_ptr(F), int(n), _ptr(axis), float(iso), _ptr(scratch), nb.value, _ptr(tris),
                                      cap, ctypes.byref(nt), _stream(stream))
        if rc == L.ERBF_ERR_CAPACITY and tri_cap is None:
            cap = nt.value
            continue
        L.check(rc)
        return tris[:nt.value]


def erbf_surface_sample(tris: torch.Tensor, u: torch.Tensor, stream=None):
    """Points, unit normals and triangle indices of area-uniform samples
    (u: float32 [S, 3] uniforms)."""
    nt, ns = tris.shape[0], u.shape[0]
    area = torch.empty(nt + (nt + 1023) // 1024, dtype=torch.float64, device=tris.device)
    pts = torch.empty((ns, 3), dtype=torch.float32, device=tris.device)
    nrm = torch.empty_like(pts)
    which = torch.empty(ns, dtype=torch.int32, device=tris.device)
    L.check(L.load().erbf_surface_sample(_ptr(tris), nt, _ptr(u), ns, _ptr(area), _ptr(pts), _ptr(nrm), _ptr(which),
                                         _stream(stream)))
    return pts, nrm, which


def erbf_surface_metrics(Pt, Nt, Pr, Nr, stream=None):
    """(HD, CD, CS) between two sampled surfaces."""
    scratch = torch.empty(2 * (Pt.shape[0] + Pr.shape[0]), dtype=torch.float64, device=Pt.device)
    out = torch.empty(3, dtype=torch.float64, device=Pt.device)
    L.check(L.load().erbf_surface_metrics(_ptr(Pt), _ptr(Nt), Pt.shape[0], _ptr(Pr), _ptr(Nr), Pr.shape[0],
                                          _ptr(scratch), _ptr(out), _stream(stream)))
    hd, cd, cs = out.cpu().tolist()
    return hd, cd, cs


def erbf_surface_metrics_noalloc(Pt, Nt, Pr, Nr, out=None, stream=None):
    """(HD, CD, CS) as erbf_surface_metrics, with the library's built-in
    scratch (nothing allocated on the device but `out` when not given)."""
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=Pt.device)
    L.check(L.load().erbf_surface_metrics_noalloc(_ptr(Pt), _ptr(Nt), Pt.shape[0], _ptr(Pr), _ptr(Nr), Pr.shape[0],
                                                  _ptr(out), _stream(stream)))
    hd, cd, cs = out.cpu().tolist()
    return hd, cd, cs


def sched_cfg(k_l2=10, tau_l2=0.5, k_l1=50, tau_l1=5.0, tau_d=0.01, T_e=1600, M_e=2000, lr0=0.01,
              lr_final=1e-3, lr_min=1e-5, refine_epochs=(400, 800)):
    """Algorithm 3's constants (defaults: the paper's values)."""
    ep = (ctypes.c_int32 * 4)(*(list(refine_epochs) + [0] * (4 - len(refine_epochs))))
    return L.SchedCfg(int(k_l2), float(tau_l2), int(k_l1), float(tau_l1), float(tau_d), int(T_e), int(M_e),
                      float(lr0), float(lr_final), float(lr_min), ep)


class SchedState:
    """Device arrays of the training-control state of every shape of a
    context (see erbf_sched_state in include/erbf.h)."""

    # the last row's first entry is the hold word (erbf_sched_state.hold)
    FLAG_ROWS = ("epoch", "l1_active", "final_phase", "add_request", "refine_request", "b_f", "n_pruned", "hold")

    def __init__(self, ctx: "Context", cfg):
        dev, n = ctx.device, ctx.n_shapes
        i32 = dict(dtype=torch.int32, device=dev)
        # the integer fields are rows of one block, so that a driver can read
        # them all with one copy (rows in FLAG_ROWS order)
        self.flags = torch.zeros((len(self.FLAG_ROWS), n), **i32)
        for i, f in enumerate(self.FLAG_ROWS):
            setattr(self, f, self.flags[i])
        self.lr = torch.zeros(n, dtype=torch.float32, device=dev)
        self.l2_ring = torch.zeros(n * cfg.k_l2, dtype=torch.float64, device=dev)
        self.bf_ring = torch.zeros(n * cfg.k_l1, **i32)
        # the hold word (erbf_sched_state.hold, the first entry of its row):
        # `c` leaves it out (every call acts), `c_hold` passes it (a call
        # with a request to act on holds the next ones)
        ptrs = {f: _ptr(getattr(self, f)) for f, _ in L.SchedState._fields_}
        self.c_hold = L.SchedState(**ptrs)
        ptrs["hold"] = None
        self.c = L.SchedState(**ptrs)
