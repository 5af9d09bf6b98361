"""The oracle's culled step at full problem sizes, spread over worker
processes.

The forward f, the cull-boundary allowance and the pair counts are sums of
per-kernel terms (eq. 3-7 with the cull of eq. 3-15-1), and each kernel's
gradient depends only on that kernel and the upstream G (Appendix A).  So the
kernels are split into chunks, each chunk runs the oracle's own functions in
a forked worker, and the parent adds the per-chunk fields and stacks the
per-kernel gradients.  The loss, the mask and the weights of eq. 3-21 are
then the oracle's functions on the whole.  Nothing here does arithmetic of
the method beyond those sums.
"""

import multiprocessing as mp
import os
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

import oracle as O

_STATE = {}


def _limit_threads():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _fwd_chunk(idx):
    olv, K = _STATE["levels"], _STATE["K"]
    Kc = O.subset(K, idx)
    f = O.forward(olv, Kc)
    allow, n_amb = O.boundary_allowance(olv, Kc) if _STATE["allow"] else (None, 0)
    return f, allow, n_amb


def _bwd_chunk(idx):
    olv, K, G = _STATE["levels"], _STATE["K"], _STATE["G"]
    Kc = O.subset(K, idx)
    gr = O.backward(olv, Kc, G)
    pf, pb = O.pair_counts(olv, Kc, G)
    return idx, gr, pf, pb


def workers() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunks(m: int, n_chunks: int):
    # interleaved chunks even out the per-kernel cost (scales vary with index)
    return [np.arange(c, m, n_chunks) for c in range(n_chunks) if c < m]


def _run(fn, items, n_proc):
    if n_proc == 1:
        _limit_threads()
        for it in items:
            yield fn(it)
        return
    ctx = mp.get_context("fork")
    with ctx.Pool(n_proc, initializer=_limit_threads) as pool:
        for out in pool.imap_unordered(fn, items):
            yield out


def forward(levels: List[O.OLevel], K: O.Kernels, allowance: bool = True, n_proc: Optional[int] = None):
    """(f per level, boundary allowance per level or None, ambiguous pair count)."""
    n_proc = n_proc or workers()
    _STATE.update(levels=levels, K=K, allow=allowance)
    f = [np.zeros(lv.npts) for lv in levels]
    al = [np.zeros(lv.npts) for lv in levels] if allowance else None
    n_amb = 0
    try:
        for fc, ac, nc in _run(_fwd_chunk, _chunks(K.m, 2 * n_proc), n_proc):
            for li in range(len(levels)):
                f[li] += fc[li]
                if allowance:
                    al[li] += ac[li]
            n_amb += nc
    finally:
        _STATE.clear()
    return f, al, n_amb


def backward(levels: List[O.OLevel], K: O.Kernels, G: List[np.ndarray], n_proc: Optional[int] = None):
    """(Grads over all kernels, P_fwd, P_bwd)."""
    n_proc = n_proc or workers()
    _STATE.update(levels=levels, K=K, G=G)
    m = K.m
    gw, ga = np.zeros(m), np.zeros(m)
    gc, gs, gq = np.zeros((m, 3)), np.zeros((m, 3)), np.zeros((m, 4))
    pf = pb = 0
    try:
        for idx, gr, pfc, pbc in _run(_bwd_chunk, _chunks(m, 2 * n_proc), n_proc):
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
