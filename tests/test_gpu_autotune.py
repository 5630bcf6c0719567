"""The autotuner against an exhaustive sweep of its search space.

The tuner times candidates in two stages (list skin x cell division with the
current force kernel, then block size x windows at the kept list
parameters), so it tries far fewer than the whole product.  Here every
combination of the four axes is timed the same way on one N = 32,000 liquid
(density 1.2, T = 0.5: the mid-size Kob-Andersen system of Sec. VI), and the
tuner's pick must run within 3% of the fastest of them."""
import statistics
import sys
import time

import pytest

from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

SKINS = (0.2, 0.25, 0.3, 0.35, 0.4, 0.5)
WG = (256, 128, 64)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _liquid():
    wl = W.ka_medium()
    r = wl.replicas[0]
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="mixed_fixed", dt=wl.dt, skin=0.3,
                  init="rsa", min_dist=0.8)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(1500, md.NVT_STOCHASTIC, n_reassign=50)
    return s


def _time(s, blob, skin, div, win, wg, steps=200, reps=5):
    """Median wall time per step of `steps` eager NVE steps from `blob`."""
    md.md_set_force_kernel(s.ctx, win, wg)
    s.set_list_params(skin, div)
    md.md_set_state(s.ctx, blob)
    s.step_nve(steps // 4)
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        s.step_nve(steps)  # syncs once at the end
        t.append((time.perf_counter() - t0) / steps)
    assert s.status() == 0
    return statistics.median(t)


def test_autotune_pick_within_3_percent_of_the_exhaustive_sweep():
    """The minimum of 72 noisy timings is biased low, so the sweep only
    nominates: its four fastest candidates and the tuner's pick are then timed
    again in alternation, three rounds, and the pick's median over the rounds
    must be within 3% of the best median among them."""
    log("case autotune vs exhaustive sweep, N=32000")
    s = _liquid()
    blob = md.md_get_state(s.ctx)
    pick = s.autotune(50)
    log(f"  pick {pick}")
    assert pick["skin"] in SKINS and pick["cell_div"] in (1, 2)
    assert pick["windows"] in (0, 1) and pick["wg_size"] in WG
    st = md.md_stats(s.ctx)
    assert (st["skin"], st["cell_div"], st["windows"], st["wg_size"]) == \
        (pick["skin"], pick["cell_div"], pick["windows"], pick["wg_size"])
    times = {}
    for skin in SKINS:
        for div in (1, 2):
            for win in (0, 1):
                for wg in WG:
                    times[(skin, div, win, wg)] = _time(s, blob, skin, div, win, wg)
    key = (pick["skin"], pick["cell_div"], pick["windows"], pick["wg_size"])
    finalists = sorted(times, key=times.get)[:4]
    if key not in finalists:
        finalists.append(key)
    rounds = {k: [] for k in finalists}
    for _ in range(3):
        for k in finalists:
            rounds[k].append(_time(s, blob, *k))
    med = {k: statistics.median(v) for k, v in rounds.items()}
    best = min(med, key=med.get)
    for k in finalists:
        log(f"  {k}: sweep {times[k] * 1e3:.4f}, rounds {' '.join(f'{t * 1e3:.4f}' for t in rounds[k])} ms/step")
    log(f"  best {best} {med[best] * 1e3:.4f}; pick {key} {med[key] * 1e3:.4f} ms/step")
    assert med[key] <= 1.03 * med[best]
    s.close()
