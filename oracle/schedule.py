"""Float64 reference of the training control of Algorithm 3 (test
infrastructure only, like the rest of this package).

After each full-batch step ("epoch" e = 1, 2, ...) the controller

1. records L2 of the step and the number of effective basis functions
   b_f = #{j : |w_j| >= tau_d} (eq. add_activate) after the update;
2. outside the final phase, in the order of Algorithm 3:
   a. prunes kernels with |w| < tau_d (eq. 3-27) when e % k_l2 == 0, L1
      is active and e < T_e;
   b. turns L1 on when e >= k_l2 and the standard deviation of the last k_l2
      L2 values is below tau_l2 (eq. l1_activate);
   c. when L1 is on, e >= k_l1 and max - min of the last k_l1 b_f values is
      below tau_l1 (eq. add_activate), requests new kernels (Algorithm 2,
      eq. 3-24) and turns L1 off;
3. at e == T_e enters the final phase: L1 off for good, no pruning or
   adding, learning rate from lr_final down to lr_min by cosine annealing
   over [T_e, M_e];
4. requests the next grid level after the epochs listed in refine_epochs
   (eq. 3-16).

Readings (the paper leaves them open): the standard deviation is the
population one (divisor k_l2); b_f is taken after the step's update and
before pruning; the learning rate of step e + 1 in the final phase is
lr_min + (lr_final - lr_min) (1 + cos(pi (e + 1 - T_e) / (M_e - T_e))) / 2.
"""

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class ScheduleConfig:
    k_l2: int = 10
    tau_l2: float = 0.5
    k_l1: int = 50
    tau_l1: float = 5.0
    tau_d: float = 0.01
    T_e: int = 1600
    M_e: int = 2000
    lr0: float = 0.01
    lr_final: float = 1e-3
    lr_min: float = 1e-5
    refine_epochs: tuple = (400, 800)


@dataclass
class ScheduleState:
    epoch: int = 0
    l1_optim: bool = False
    final_phase: bool = False
    add_request: bool = False
    refine_request: bool = False
    prune_now: bool = False
    b_f: int = 0
    lr: float = 0.01
    l2_hist: List[float] = field(default_factory=list)
    bf_hist: List[int] = field(default_factory=list)


def effective_count(w: np.ndarray, tau_d: float) -> int:
    """b_f of eq. add_activate."""
    return int(np.count_nonzero(np.abs(np.asarray(w, np.float64)) >= tau_d))


def final_lr(cfg: ScheduleConfig, e: int) -> float:
    frac = min(max((e - cfg.T_e) / float(cfg.M_e - cfg.T_e), 0.0), 1.0)
    return cfg.lr_min + 0.5 * (cfg.lr_final - cfg.lr_min) * (1.0 + math.cos(math.pi * frac))


def control_step(st: ScheduleState, cfg: ScheduleConfig, l2: float, w: np.ndarray) -> ScheduleState:
    """Algorithm 3's bookkeeping after one step; returns the new state.
    `prune_now` says whether eq. 3-27 is to be applied to this step's
    parameters (see :func:`prune`)."""
    s = ScheduleState(**{k: (list(v) if isinstance(v, list) else v) for k, v in st.__dict__.items()})
    s.epoch = e = st.epoch + 1
    s.add_request = s.refine_request = s.prune_now = False
    s.b_f = effective_count(w, cfg.tau_d)
    s.l2_hist = (s.l2_hist + [float(l2)])[-cfg.k_l2:]
    s.bf_hist = (s.bf_hist + [s.b_f])[-cfg.k_l1:]
    if not s.final_phase:
        if e % cfg.k_l2 == 0 and s.l1_optim and e < cfg.T_e:
            s.prune_now = True
        if not s.l1_optim and e >= cfg.k_l2 and float(np.std(s.l2_hist)) < cfg.tau_l2:
            s.l1_optim = True
        if s.l1_optim and e >= cfg.k_l1 and (max(s.bf_hist) - min(s.bf_hist)) < cfg.tau_l1:
            s.add_request = True
            s.l1_optim = False
    if e == cfg.T_e:
        s.final_phase = True
        s.l1_optim = False
    if e in cfg.refine_epochs:
        s.refine_request = True
    s.lr = final_lr(cfg, e + 1) if s.final_phase else cfg.lr0
    return s


def prune(p: np.ndarray, m: int, cap: int, tau_d: float, *moments):
    """eq. 3-27: keep the kernels with |w| >= tau_d, in their order.  Returns
    the new packed parameters, the new count and the moments compacted the
    same way (slots past the new count are zero)."""
    P = np.asarray(p, np.float64).reshape(11, cap)
    keep = np.abs(P[0, :m]) >= tau_d
    idx = np.nonzero(keep)[0]
    out = []
    for arr in (P,) + tuple(np.asarray(x, np.float64).reshape(11, cap) for x in moments):
        n = np.zeros_like(arr)
        n[:, :idx.size] = arr[:, idx]
        out.append(n.reshape(-1))
    return (out[0], int(idx.size)) + tuple(out[1:])
