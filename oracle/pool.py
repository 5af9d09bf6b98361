"""The oracle's culled step at full problem sizes, spread over worker
processes.  Test infrastructure, like the rest of the oracle: only the tests,
the smoke check and the benchmark's CPU baseline use it.

The forward f, the cull-boundary allowance and the pair counts are sums of
per-kernel terms (eq. 3-7 with the cull of eq. 3-15-1), and each kernel's
gradient depends only on that kernel and the upstream G (Appendix A).  So the
kernels are split into chunks, each chunk runs the oracle's own functions in
a worker process, and the parent adds the per-chunk fields and stacks the
per-kernel gradients.  The loss, the mask and the weights of eq. 3-21 are
then the oracle's functions on the whole.  Nothing here does arithmetic of
the method beyond those sums.

Workers come from a fork server (multiprocessing's "forkserver" start
method): a clean process started once, early, that forks the workers, so no
worker is a copy of a caller that has already used the GPU or carries a
profiler's state.  Call start_server() before anything touches the GPU; the
problem is handed to each worker once, at its start.
"""

import multiprocessing as mp
import os
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import erbf as O

_STATE = {}
_CTX = "forkserver"


def start_server():
    """Start the fork server now (before the caller initialises the GPU)."""
    ctx = mp.get_context(_CTX)
    ctx.set_forkserver_preload(["numpy", "oracle"])
    from multiprocessing import forkserver
    forkserver.ensure_running()


def _init_worker(state):
    _limit_threads()
    _STATE.clear()
    _STATE.update(state)
    # the upstream G travels as (index, value) pairs of its non-zero entries
    if "G_sparse" in _STATE:
        G = []
        for n, (ix, v) in zip(_STATE["npts"], _STATE.pop("G_sparse")):
            g = np.zeros(n)
            g[ix] = v
            G.append(g)
        _STATE["G"] = G


def _limit_threads():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _span(*arrays):
    """[lo, hi) holding every non-zero entry of the arrays (None when all 0)."""
    nz = [np.flatnonzero(a) for a in arrays if a is not None]
    nz = [z for z in nz if z.size]
    if not nz:
        return None
    return int(min(z[0] for z in nz)), int(max(z[-1] for z in nz)) + 1


def _fwd_chunk(idx):
    olv, K = _STATE["levels"], _STATE["K"]
    Kc = O.subset(K, idx)
    f = O.forward(olv, Kc)
    allow, n_amb = O.boundary_allowance(olv, Kc) if _STATE["allow"] else (None, 0)
    # a chunk of neighbouring kernels touches a slab of each level: return f
    # at the active points of the span of its non-zero entries, and the
    # (sparse) allowance as (index, value) pairs
    out = []
    for li, lv in enumerate(olv):
        sp = _span(f[li], allow[li] if allow is not None else None)
        if sp is None:
            out.append(None)
            continue
        lo, hi = sp
        act = lv.act()[lo:hi]
        av = None
        if allow is not None:
            ix = np.flatnonzero(allow[li][lo:hi])
            av = (ix, allow[li][lo:hi][ix])
        out.append((lo, hi, f[li][lo:hi][act], av))
    return out, n_amb


def _bwd_chunk(idx):
    olv, K, G = _STATE["levels"], _STATE["K"], _STATE["G"]
    Kc = O.subset(K, idx)
    gr = O.backward(olv, Kc, G)
    pf, pb = O.pair_counts(olv, Kc, G)
    return idx, gr, pf, pb


def workers() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunks(K: O.Kernels, n_chunks: int):
    """Contiguous runs of the kernels ordered by centre (z, then y, then x),
    so that each chunk's field is confined to a slab; many more chunks than
    workers even out the per-kernel cost."""
    m = K.m
    order = np.lexsort((K.c[:, 0], K.c[:, 1], K.c[:, 2])) if m else np.zeros(0, np.int64)
    return [c for c in np.array_split(order, min(n_chunks, m)) if c.size] if m else []


def _run(fn, items, n_proc):
    if n_proc == 1:
        _limit_threads()
        for it in items:
            yield fn(it)
        return
    ctx = mp.get_context(_CTX)
    with ctx.Pool(n_proc, initializer=_init_worker, initargs=(dict(_STATE),)) as pool:
        for out in pool.imap_unordered(fn, items):
            yield out


def _light(levels):
    """The levels as the workers need them: grid axes and masks (targets and
    raw distances stay behind), sample sets whole."""
    return [lv if isinstance(lv, O.OSamples) else O.OLevel(lv.n, lv.axis, lv.active) for lv in levels]


def forward(levels: List[O.OLevel], K: O.Kernels, allowance: bool = True, n_proc: Optional[int] = None):
    """(f per level, boundary allowance per level or None, ambiguous pair count)."""
    n_proc = n_proc or workers()
    _STATE.update(levels=_light(levels) if n_proc > 1 else levels, K=K, allow=allowance)
    f = [np.zeros(lv.npts) for lv in levels]
    al = [np.zeros(lv.npts) for lv in levels] if allowance else None
    n_amb = 0
    try:
        acts = [lv.act() for lv in levels]
        for parts, nc in _run(_fwd_chunk, _chunks(K, 8 * n_proc), n_proc):
            for li, part in enumerate(parts):
                if part is None:
                    continue
                lo, hi, fv, av = part
                seg = f[li][lo:hi]
                seg[acts[li][lo:hi]] += fv
                if allowance:
                    al[li][lo + av[0]] += av[1]
            n_amb += nc
    finally:
        _STATE.clear()
    return f, al, n_amb


def backward(levels: List[O.OLevel], K: O.Kernels, G: List[np.ndarray], n_proc: Optional[int] = None):
    """(Grads over all kernels, P_fwd, P_bwd)."""
    n_proc = n_proc or workers()
    if n_proc > 1:
        Gs = []
        for g in G:
            ix = np.flatnonzero(g)
            Gs.append((ix, np.asarray(g)[ix]))
        _STATE.update(levels=_light(levels), K=K, G_sparse=Gs, npts=[lv.npts for lv in levels])
    else:
        _STATE.update(levels=levels, K=K, G=G)
    m = K.m
    gw, ga = np.zeros(m), np.zeros(m)
    gc, gs, gq = np.zeros((m, 3)), np.zeros((m, 3)), np.zeros((m, 4))
    pf = pb = 0
    try:
        for idx, gr, pfc, pbc in _run(_bwd_chunk, _chunks(K, 8 * n_proc), n_proc):
            gw[idx], ga[idx], gc[idx], gs[idx], gq[idx] = gr.w, gr.a, gr.c, gr.s, gr.q
            pf += pfc
            pb += pbc
    finally:
        _STATE.clear()
    return O.Grads(gw, gc, gs, gq, ga), pf, pb


@dataclass
class FullStep:
    f: List[np.ndarray]
    allow: List[np.ndarray]
    n_amb: int
    loss: O.LossOut
    G: List[np.ndarray]
    grads_l2: O.Grads
    alpha: float
    beta: float
    grads: O.Grads
    P_fwd: int
    P_bwd: int


def step(levels, K, mode=O.MODE_FIXED, lam=0.0, l1_active=False, tau1=0.9, tau2=1.1, tau_m=0.02,
         n_proc=None) -> FullStep:
    """The oracle's step (forward, eq. 3-18/3-19 loss, backward, eq. 3-21)."""
    f, al, n_amb = forward(levels, K, True, n_proc)
    lo = O.loss(levels, f, K, tau1, tau2)
    G = [2.0 * e for e in lo.E]
    gr, pf, pb = backward(levels, K, G, n_proc)
    a, b = O.loss_weights(mode, lam, l1_active, lo.max_abs_E, tau_m, gr.w, K.w)
    return FullStep(f, al, n_amb, lo, G, gr, a, b, O.combine(gr, K.w, a, b), pf, pb)
