"""Temperature-ladder run sequence on the batched engine (Sec. V, and the
mean-square-displacement exercise of the appendix).

Each stage takes the configuration the previous stage ended with, applies
the bath at the stage temperature for ``n_equil`` steps, optionally rescales
the velocities so that the total energy equals the bath run's time-averaged
total energy (the paper's recommendation for the Nose-Hoover bath at low
temperature), continues with ``n_equil`` NVE steps, and then runs ``n_prod``
NVE production steps during which the mean-square displacement of each
species is measured at log-spaced steps (``md_log_schedule``).  Every
replica of the system is an independent ladder (the paper's eight
independent initial configurations are eight replicas), so all ladders
advance in one launch per kernel.

The diffusion constant of species a follows from the long-time form
<r_a^2(t)> = 2 d D_a t with d = 3 (Eq. (msd6Dt)), fitted by least squares
(with an intercept, which absorbs the short-time ballistic part) over the
late part of the production run.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import md


@dataclass
class Stage:
    temperature: float
    n_equil: int
    n_prod: int


@dataclass
class StageResult:
    temperature: float
    times: np.ndarray            # [K] measurement times (steps * dt)
    msd: np.ndarray              # [K][n_rep][2] MSD of A and B against the production start
    diffusion: np.ndarray        # [n_rep][2] fitted D_A, D_B
    fit_from: float              # first time used by the fit
    energy_target: Optional[np.ndarray] = None  # [n_rep] E_tot the velocities were scaled to
    observables_end: np.ndarray = field(default_factory=lambda: np.zeros(0))  # [n_rep][6]


def diffusion_fit(t, msd, t_from: float, dim: int = 3):
    """Least-squares fit of msd = 2 dim D t + c over t >= t_from.  t: [K];
    msd: [K] or [K, ...].  Returns (D, c) with the trailing shape of msd."""
    t = np.asarray(t, np.float64)
    y = np.asarray(msd, np.float64)
    sel = t >= t_from
    if np.count_nonzero(sel) < 2:
        raise ValueError("diffusion_fit needs at least two times at or after t_from")
    ts = t[sel]
    ys = y[sel].reshape(ts.size, -1)
    A = np.stack([ts, np.ones_like(ts)], axis=1)
    coef, *_ = np.linalg.lstsq(A, ys, rcond=None)
    D = coef[0] / (2.0 * dim)
    c = coef[1]
    return D.reshape(y.shape[1:]), c.reshape(y.shape[1:])


def _bath(system, n, mode, n_reassign, tau):
    if n <= 0:
        return
    if mode == md.NVT_STOCHASTIC:
        system.step_nvt(n, md.NVT_STOCHASTIC, n_reassign=n_reassign)
    else:
        system.step_nvt(n, md.NVT_NOSE_HOOVER, tau=tau)


def run_stage(system, stage: Stage, dt: float, mode: int = md.NVT_STOCHASTIC, n_reassign: int = 50,
              tau: float = 0.5, rescale_energy: bool = False, average_last: float = 0.25,
              samples: int = 20, t0: float = 1.0, kmax: int = 60, fit_decades: float = 1.0) -> StageResult:
    """One rung of the ladder on every replica of ``system`` (an md.System)."""
    system.set_temperature(stage.temperature)
    target = None
    if rescale_energy:
        # bath run; E_tot averaged over `samples` points spread over its last part
        n_avg = max(1, int(round(stage.n_equil * average_last)))
        _bath(system, stage.n_equil - n_avg, mode, n_reassign, tau)
        k = max(1, min(samples, n_avg))
        chunks = np.diff(np.linspace(0, n_avg, k + 1).round().astype(int))
        e = []
        for c in chunks:
            _bath(system, int(c), mode, n_reassign, tau)
            e.append(system.observables()[:, 4])
        target = np.mean(e, axis=0)
        obs = system.observables()
        ke, pe = obs[:, 0], obs[:, 1]
        want = target - pe
        if np.any(want <= 0.0):
            raise RuntimeError("energy rescale: target total energy below the potential energy")
        system.scale_velocities(np.sqrt(want / ke))
    else:
        _bath(system, stage.n_equil, mode, n_reassign, tau)
    if stage.n_equil > 0:
        system.step_nve(stage.n_equil)
    steps = md.md_log_schedule(stage.n_prod, t0, kmax)
    system.msd_set_origin(0)
    rows, prev = [], 0
    for st in steps:
        system.step_nve(int(st) - prev)
        prev = int(st)
        rows.append(system.msd(0))
    msd = np.array(rows)
    times = steps.astype(np.float64) * dt
    t_from = times[-1] / (10.0 ** fit_decades)
    D, _ = diffusion_fit(times, msd, t_from)
    return StageResult(stage.temperature, times, msd, D, t_from, target, system.observables())


def run_ladder(system, stages: List[Stage], dt: float, **kw) -> List[StageResult]:
    """All rungs in order; each starts from the configuration the previous one ended with."""
    return [run_stage(system, st, dt, **kw) for st in stages]
