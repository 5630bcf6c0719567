"""Statistical comparison of trajectories.

The dynamics are chaotic: an MIXED or MIXED_FIXED run and an FP64 run from the
same state part after some hundred steps, so they are compared by the
averages the paper measures, not step by step:

  - the time-averaged pair-distance histogram (Sec. VI.A.1; g_ab(r) of Eqs.
    (gAA), (gAB) up to a fixed normalisation) in windows over the first
    peaks and the first minimum of AA, AB and BB;
  - the mean-square displacement (Eqs. (msdwithi), (msdtw)) of A and B at
    lags of 10, 100 and 1000 steps, averaged over five time origins;

each within five combined standard errors (block averages) plus a 1%
floor.  And the stochastic bath (Sec. II.E.1) holds the mean temperature
(Eq. (equip3N)) at its target.  The FP64 path itself is pinned to the oracle
step by step in the other GPU tests.  Workload: N = 4000, density 1.2,
T = 1.0 (a liquid that decorrelates in a few hundred steps).
"""
import math
import sys

import numpy as np
import pytest

from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

N, RHO, T = 4000, 1.2, 1.0
STEPS, CHUNK = 6000, 10
RDF_EVERY, BLOCKS = 100, 6
ORIGINS = (0, 1000, 2000, 3000, 4000)
LAGS = (10, 100, 1000)
DR, NBINS = 0.02, 150  # r up to 3.0
WINDOWS = {  # (pair row, r_lo, r_hi): first peaks and the AA first minimum
    "AA peak": (0, 0.95, 1.25), "AB peak": (1, 0.78, 1.05), "BB peak": (2, 0.85, 1.15),
    "AA minimum": (0, 1.30, 1.70),
}
_STATE = {}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def start():
    """One equilibrated state (FP64 stochastic bath), shared by every run."""
    if "x" not in _STATE:
        L = W.box_for(N, RHO)
        s = md.System([(N, W.n_a_for(N), L, T, 51)], precision="fp64", init="rsa", min_dist=0.8, skin=0.3)
        s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
        s.step_nvt(1500, md.NVT_STOCHASTIC, n_reassign=50)
        s.sync()
        a = s.numpy(("x", "y", "z", "vx", "vy", "vz"))
        assert s.status() == 0
        s.close()
        _STATE.update(a)
        _STATE["L"] = L
    return _STATE


def run(prec):
    st = start()
    L = st["L"]
    s = md.System([(N, W.n_a_for(N), L, T, 51)], precision=prec, skin=0.3,
                  positions=(st["x"], st["y"], st["z"]), velocities=(st["vx"], st["vy"], st["vz"]),
                  msd_slots=len(ORIGINS))
    hists, msd = [], {}
    for t in range(0, STEPS + 1, CHUNK):
        if t in ORIGINS:
            s.msd_set_origin(ORIGINS.index(t))
        for k, o in enumerate(ORIGINS):
            if t - o in LAGS:
                msd[(k, t - o)] = s.msd(k)[0]
        if t % RDF_EVERY == 0 and t > 0:
            hists.append(s._host(s.rdf(DR, NBINS))[0].astype(np.float64))
        if t < STEPS:
            s.step_nve(CHUNK)
    assert s.status() == 0
    s.close()
    return np.array(hists), msd


def window_fractions(h):
    """Per sample: the fraction of each pair row's counts inside each window."""
    r = (np.arange(NBINS) + 0.5) * DR
    out = {}
    for name, (row, lo, hi) in WINDOWS.items():
        m = (r >= lo) & (r < hi)
        out[name] = h[:, row, m].sum(1) / h[:, row, :].sum(1)
    return out


def mean_se(v, blocks):
    b = np.array([x.mean() for x in np.array_split(np.asarray(v), blocks)])
    return b.mean(), b.std(ddof=1) / math.sqrt(blocks)


@pytest.fixture(scope="module")
def fp64_run():
    return run("fp64")


def agree(name, a, b):
    (ma, sa), (mb, sb) = a, b
    bound = 5.0 * math.hypot(sa, sb) + 0.01 * abs(mb)
    log(f"  {name}: {ma:.6g} +- {sa:.2g} vs FP64 {mb:.6g} +- {sb:.2g} (bound {bound:.3g})")
    assert abs(ma - mb) <= bound, name


@pytest.mark.parametrize("prec", ["mixed", "mixed_fixed"])
def test_rdf_and_msd_statistics_match_fp64(prec, fp64_run):
    log(f"case statistics {prec} vs fp64, N={N}, T={T}, {STEPS} NVE steps")
    h, msd = run(prec)
    h0, msd0 = fp64_run
    assert len(h) == len(h0) == STEPS // RDF_EVERY
    f, f0 = window_fractions(h), window_fractions(h0)
    for name in WINDOWS:
        agree(name, mean_se(f[name], BLOCKS), mean_se(f0[name], BLOCKS))
    for lag in LAGS:
        for sp, label in ((0, "A"), (1, "B")):
            v = [msd[(k, lag)][sp] for k in range(len(ORIGINS))]
            v0 = [msd0[(k, lag)][sp] for k in range(len(ORIGINS))]
            agree(f"MSD_{label}({lag} steps)", mean_se(v, len(v)), mean_se(v0, len(v0)))


def test_stochastic_bath_holds_the_target_temperature():
    """Mean temperature of the sampled rows over 3000 bath steps (redraw every
    50) after a 500-step start: within 1% of T (one sample fluctuates by about
    sqrt(2 / 3N) = 1.3%)."""
    log(f"case bath temperature N={N}, T={T}")
    L = W.box_for(N, RHO)
    s = md.System([(N, W.n_a_for(N), L, T, 61)], precision="mixed_fixed", init="rsa", min_dist=0.8, skin=0.3,
                  sample_every=10, sample_capacity=400)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.clear_samples()
    s.step_nvt(3000, md.NVT_STOCHASTIC, n_reassign=50)
    rows = s.samples()[0]
    assert s.status() == 0
    s.close()
    temps = rows[:, 4]
    m, se = mean_se(temps, 10)
    log(f"  <T> = {m:.5f} +- {se:.2g} over {len(temps)} samples")
    assert len(temps) == 300
    assert abs(m - T) <= 0.01 * T
