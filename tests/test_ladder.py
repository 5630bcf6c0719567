"""Host logic of the temperature ladder: the diffusion fit and the order of
operations of one rung, with a recording stand-in for the GPU system."""
import numpy as np
import pytest

from paper_2001_07089_amd import ladder, md


def test_diffusion_fit_recovers_linear_regime():
    t = np.geomspace(0.005, 50.0, 80)
    D = np.array([0.031, 0.057])
    # ballistic start (3 T t^2 with T = 1) joined to the diffusive line
    lin = 6.0 * D[None, :] * t[:, None] + 0.4
    msd = np.where(t[:, None] < 1.0, 3.0 * t[:, None] ** 2, lin)
    got, c = ladder.diffusion_fit(t, msd, t_from=5.0)
    assert np.allclose(got, D, rtol=1e-12) and np.allclose(c, 0.4, rtol=1e-10)
    # one-dimensional input, 2-d fit
    got2, _ = ladder.diffusion_fit(t, 4.0 * 0.2 * t, t_from=1.0, dim=2)
    assert got2 == pytest.approx(0.2, rel=1e-12)
    with pytest.raises(ValueError):
        ladder.diffusion_fit(t, msd, t_from=1e9)


class FakeSystem:
    """Records the calls run_stage makes; KE/PE chosen by the test."""

    def __init__(self, n_rep, ke, pe, e_series):
        self.n_rep = n_rep
        self.calls = []
        self.ke, self.pe = np.array(ke, float), np.array(pe, float)
        self.e_series = list(e_series)
        self.t = 0

    def set_temperature(self, T):
        self.calls.append(("T", T))

    def step_nvt(self, n, mode, n_reassign=None, tau=None):
        self.calls.append(("nvt", n))
        self.t += n

    def step_nve(self, n):
        self.calls.append(("nve", n))
        self.t += n

    def observables(self):
        out = np.zeros((self.n_rep, 6))
        out[:, 0], out[:, 1] = self.ke, self.pe
        out[:, 4] = self.e_series.pop(0) if self.e_series else self.ke + self.pe
        return out

    def scale_velocities(self, f):
        self.calls.append(("scale", np.array(f)))

    def msd_set_origin(self, slot):
        self.calls.append(("origin", slot))
        self.t0 = self.t

    def msd(self, slot):
        dt = (self.t - self.t0) * 0.005
        return np.tile([[6 * 0.05 * dt, 6 * 0.08 * dt]], (self.n_rep, 1))


def test_run_stage_sequence_and_energy_rescale():
    e_series = [[-5.0, -6.0]] * 4 + [[-5.2, -6.2]] * 4  # averaged: -5.1, -6.1
    fs = FakeSystem(2, ke=[1.0, 2.0], pe=[-6.5, -7.9], e_series=e_series)
    st = ladder.Stage(temperature=0.8, n_equil=800, n_prod=1000)
    res = ladder.run_stage(fs, st, 0.005, rescale_energy=True, average_last=0.25, samples=8)
    assert fs.calls[0] == ("T", 0.8)
    nvt = sum(c[1] for c in fs.calls if c[0] == "nvt")
    assert nvt == 800
    scale = [c[1] for c in fs.calls if c[0] == "scale"][0]
    assert np.allclose(scale, np.sqrt((np.array([-5.1, -6.1]) - np.array([-6.5, -7.9])) / np.array([1.0, 2.0])))
    assert np.allclose(res.energy_target, [-5.1, -6.1])
    nve = [c[1] for c in fs.calls if c[0] == "nve"]
    assert nve[0] == 800 and sum(nve[1:]) == 1000  # equilibration, then the log-spaced production
    steps = np.cumsum(nve[1:])
    assert np.array_equal(steps, md.md_log_schedule(1000, 1.0, 60))
    assert np.allclose(res.diffusion, [[0.05, 0.08]] * 2, rtol=1e-9)
    assert res.fit_from == pytest.approx(res.times[-1] / 10)


def test_run_ladder_without_rescale_keeps_velocities():
    fs = FakeSystem(1, ke=[1.0], pe=[-6.0], e_series=[])
    out = ladder.run_ladder(fs, [ladder.Stage(2.0, 100, 200), ladder.Stage(1.0, 100, 200)], 0.005)
    assert [r.temperature for r in out] == [2.0, 1.0]
    assert not any(c[0] == "scale" for c in fs.calls)
    assert [c for c in fs.calls if c[0] == "T"] == [("T", 2.0), ("T", 1.0)]


class FakeAgingSystem(FakeSystem):
    def __init__(self):
        super().__init__(1, ke=[1.0], pe=[-6.0], e_series=[])
        self.origins = {}

    def msd_set_origin(self, slot):
        self.calls.append(("origin", slot, self.t))
        self.origins[slot] = self.t

    def msd(self, slot):
        return np.array([[float(self.t - self.origins[slot]), 0.0]])


def test_quench_schedule_per_waiting_time():
    from paper_2001_07089_amd import aging
    fs = FakeAgingSystem()
    out = aging.quench(fs, 0.3, 1000, t_w=(0, 10, 100, 500))
    assert fs.calls[0] == ("T", 0.3)
    origins = [c for c in fs.calls if c[0] == "origin"]
    assert [(c[1], c[2]) for c in origins] == [(0, 0), (1, 10), (2, 100), (3, 500)]
    assert sum(c[1] for c in fs.calls if c[0] == "nvt") == 1000
    for tw, cur in out.items():
        assert np.array_equal(cur.lags, md.md_log_schedule(1000 - tw, 1.0, 60))
        # each recorded value is the lag itself (the stand-in's MSD is t - t_origin)
        assert np.array_equal(cur.msd[:, 0, 0], cur.lags.astype(float))
    import pytest as _pt
    with _pt.raises(ValueError):
        aging.quench(fs, 0.3, 100, t_w=(0, 100))
