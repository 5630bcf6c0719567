"""Aging after an instant temperature quench (Sec. V; the two-time MSD
exercise of the appendix, Eq. (msdtw)).

A system equilibrated at T_i is set to T_f and continued with the bath.  At
each waiting time t_w (steps since the quench) the current unwrapped
positions become an MSD origin; the two-time mean-square displacement
<r_a^2(t_w, t_w + t)> is measured at log-spaced lags t (``md_log_schedule``)
for every origin, and, when asked, the self part of the van Hove function
at the same points.  Every replica is an independent quench.
"""
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np

from . import md


@dataclass
class AgingCurve:
    t_w: int                      # waiting time in steps
    lags: np.ndarray              # [K] lags in steps
    msd: np.ndarray               # [K][n_rep][2]
    van_hove: Optional[np.ndarray] = None  # [K][n_rep][2][n_bins] counts


def quench(system, T_final: float, n_steps: int, t_w: Sequence[int] = (0, 10, 100, 500),
           mode: int = md.NVT_STOCHASTIC, n_reassign: int = 50, tau: float = 0.5, t0: float = 1.0,
           kmax: int = 60, van_hove: Optional[tuple] = None) -> Dict[int, AgingCurve]:
    """Quench every replica of ``system`` (an md.System) to T_final and follow
    it for n_steps bath steps.  van_hove = (dr, n_bins) also records the self
    van Hove histogram at every measurement.  At most 16 waiting times."""
    t_w = sorted(int(t) for t in t_w)
    if len(t_w) > 16 or t_w[0] < 0 or t_w[-1] >= n_steps:
        raise ValueError("need at most 16 waiting times in [0, n_steps)")
    plan = {tw: md.md_log_schedule(n_steps - tw, t0, kmax) for tw in t_w}
    points = sorted(set(t_w) | {tw + int(l) for tw, lags in plan.items() for l in lags})
    lagset = {tw: set(int(l) for l in lags) for tw, lags in plan.items()}
    slot = {tw: k for k, tw in enumerate(t_w)}
    rec = {tw: [] for tw in t_w}
    vh = {tw: [] for tw in t_w}
    system.set_temperature(T_final)
    now = 0
    for p in points:
        if p > now:
            if mode == md.NVT_STOCHASTIC:
                system.step_nvt(p - now, md.NVT_STOCHASTIC, n_reassign=n_reassign)
            else:
                system.step_nvt(p - now, md.NVT_NOSE_HOOVER, tau=tau)
            now = p
        for tw in t_w:
            if tw == now:
                system.msd_set_origin(slot[tw])
            elif tw < now and (now - tw) in lagset[tw]:
                rec[tw].append(system.msd(slot[tw]))
                if van_hove is not None:
                    h = system.van_hove(slot[tw], van_hove[0], van_hove[1])
                    vh[tw].append(system._host(h).astype(np.int64))
    return {tw: AgingCurve(tw, plan[tw].astype(np.int64), np.array(rec[tw]),
                           np.array(vh[tw]) if van_hove is not None else None) for tw in t_w}

