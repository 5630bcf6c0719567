"""Sampled observables (the ring buffer of md_observables) and the NVE energy
drift measured from them.

The paper follows the kinetic, potential and total energy along a run
(Sec. III.F, Eq. (EsysNpart)) and the temperature (Eq. (equip3N)); LAMMPS
prints them every few steps (Sec. IV.B).  Rows are written on the device at
every step that is a multiple of sample_every, in eager calls and in graph
replays.  Drift follows the windowed definition: the relative change of the
500-step window means of E_tot between the first and the last window of the
run, scaled to 10^4 steps.
"""
import sys

import numpy as np
import pytest

from paper_2001_07089_amd import analysis
from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def windowed_drift(rows, window_steps=500):
    out = analysis.energy_drift(rows, window_steps)
    return out["windowed"], out["slope"]


def test_rows_match_the_instant_observables():
    n = 1000
    L = W.box_for(n, 1.2)
    s = md.System([(n, W.n_a_for(n), L, 1.0, 5)], precision="fp64", init="rsa", sample_every=10,
                  sample_capacity=64)
    s.step_nve(95)          # fused steps; samples at 10, 20, ..., 90
    s.step_nve(5)           # the last step of a call is not fused: sample at 100
    rows = s.samples()[0]
    assert rows.shape == (10, 6)
    assert np.array_equal(rows[:, 0], np.arange(10, 101, 10))
    now = s.observables()[0]           # KE, PE, W, T, E_tot, P at step 100
    last = rows[-1]
    assert last[1] == pytest.approx(now[0], rel=1e-12)
    assert last[2] == pytest.approx(now[1], rel=1e-12)
    assert last[3] == pytest.approx(now[4], rel=1e-12)
    assert last[4] == pytest.approx(now[3], rel=1e-12)
    assert last[5] == pytest.approx(now[2], rel=1e-12)
    # E_tot = KE + PE and T = 2 KE / 3N on every row
    assert np.allclose(rows[:, 3], rows[:, 1] + rows[:, 2], rtol=1e-14, atol=0)
    assert np.allclose(rows[:, 4], 2 * rows[:, 1] / (3 * n), rtol=1e-14, atol=0)
    s.clear_samples()
    assert s.samples().shape[1] == 0
    s.close()


def test_rows_inside_graph_replays_and_the_ring_wraps():
    reps = [(500, 400, W.box_for(500, 1.2), 0.8, 1), (900, 720, W.box_for(900, 1.2), 1.5, 2)]
    s = md.System(reps, precision="mixed_fixed", init="rsa", sample_every=4, sample_capacity=16)
    md.md_graph_capture(s.ctx, 40, 0)
    for _ in range(3):
        md.md_graph_launch(s.ctx)
    rows = s.samples()
    assert rows.shape == (2, 16, 6)
    assert np.array_equal(rows[0, :, 0], np.arange(120 - 15 * 4, 121, 4))   # the last 16 samples
    assert np.array_equal(rows[0, :, 0], rows[1, :, 0])
    assert np.all(rows[:, :, 1] > 0) and np.all(rows[:, :, 2] < 0)
    # the second replica is hotter
    assert rows[1, :, 4].mean() > rows[0, :, 4].mean()
    assert s.status() == 0
    s.close()


def test_sample_at_a_redraw_step_sees_the_bath_temperature():
    n, T = 2000, 0.6
    s = md.System([(n, W.n_a_for(n), W.box_for(n, 1.2), T, 9)], precision="fp64", init="rsa", sample_every=5)
    s.step_nvt(50, md.NVT_STOCHASTIC, n_reassign=10)
    rows = s.samples()[0]
    redraw = rows[rows[:, 0] % 10 == 0]
    assert len(redraw) == 5
    assert np.allclose(redraw[:, 4], T, rtol=1e-13, atol=0)
    # between redraws the temperature moves away from T
    assert np.any(np.abs(rows[rows[:, 0] % 10 == 5, 4] - T) > 1e-6)
    # Nose-Hoover steps sample too
    s.clear_samples()
    s.step_nvt(20, md.NVT_NOSE_HOOVER, tau=0.5)
    rows = s.samples()[0]
    assert np.array_equal(rows[:, 0], np.arange(55, 71, 5))
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fixed"])
def test_nve_drift_bound_at_32000(prec):
    """N = 32,000 at T = 0.5 (random sequential addition, stochastic bath),
    then 10^4 NVE steps at dt = 0.005 sampled every 10 steps: drift at most
    1e-4 per 10^4 steps by the windowed definition and by the fitted slope."""
    wl = W.ka_medium()
    r = wl.replicas[0]
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision=prec, dt=wl.dt, init="rsa",
                  auto_sync=False, sample_every=10, sample_capacity=1024)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(4500, md.NVT_STOCHASTIC, n_reassign=50)
    s.step_nve(1000)
    s.clear_samples()
    md.md_graph_capture(s.ctx, 1000, 0)
    for _ in range(10):
        md.md_graph_launch(s.ctx)
    rows = s.samples()[0]
    assert s.status() == 0
    assert rows.shape[0] == 1000
    d, slope = windowed_drift(rows)
    log(f"  {prec}: drift {d:.2e} per 1e4 steps (slope {slope:.2e}), E/N {rows[0, 3] / r.n:.5f}, "
        f"T {rows[:, 4].mean():.4f}")
    assert d <= 1e-4
    assert slope <= 1e-4
    s.close()
