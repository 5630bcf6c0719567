"""Parity of the step kernel's window variant (mixed precisions).

With windows on, a list part whose stencil rows fit is stored as 16-bit
offsets into LDS copies of those rows (in up to four groups of consecutive
rows), and its neighbours are read from LDS; the pair arithmetic and the order
of the entries are those of the direct variant, and the padding between
groups pairs a particle with its own copy, which adds exact zeros.  So the
forces, and with them whole trajectories, must equal the direct variant's bit
for bit in both mixed precisions, for every block size; the direct variant is
checked against the FP64 oracle (Eq. (KAFix)) in the other parity tests, and
here once more at N = 4000 with windows on."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _liquid(reps, precision, nvt=300, **kw):
    """Replicas (n, rho, T, seed) from RSA starts, melted by the stochastic bath."""
    rr = [(n, W.n_a_for(n), W.box_for(n, rho), T, seed) for n, rho, T, seed in reps]
    s = md.System(rr, precision=precision, init="rsa", min_dist=0.8, skin=0.3, **kw)
    s.step_nvt(nvt, md.NVT_STOCHASTIC, n_reassign=10)
    s.sync()
    return s


def _forces(s, windows, wg, energy=False):
    """Forces after a fresh list build with the given variant.  Every variant
    builds from the same positions, so the slot order (which a rebuild sets,
    and which orders the FP32 sums of MIXED) is the same for all of them."""
    md.md_set_force_kernel(s.ctx, windows, wg)
    s.build_cells()
    obs = s.forces(energy=energy)
    s.sync()
    a = s.numpy(("ax", "ay", "az"))
    assert s.status() == 0
    return a, obs


BATCH = [(4000, 1.2, 1.0, 11), (1500, 1.2, 0.6, 12), (700, 1.1, 1.5, 13), (9000, 1.3, 0.8, 14)]


@pytest.mark.parametrize("prec", ["mixed", "mixed_fixed"])
def test_window_forces_equal_direct_bit_for_bit(prec):
    log(f"case windows forces {prec}", BATCH)
    s = _liquid(BATCH, prec)
    _forces(s, 0, 256)  # one build first: the later builds keep its slot order
    ref, obs0 = _forces(s, 0, 256, energy=True)
    for wg in (256, 128, 64):
        a, obs = _forces(s, 1, wg, energy=True)
        st = md.md_stats(s.ctx)
        log(f"  wg {wg}: staged fraction {st['staged_fraction']:.3f}")
        assert st["windows"] == 1 and st["wg_size"] == wg and st["staged_fraction"] > 0.5
        for k in ref:
            assert np.array_equal(a[k], ref[k]), (wg, k)
        assert np.array_equal(obs[:, :2], obs0[:, :2])  # PE and virial
    s.close()


def test_window_forces_match_oracle():
    log("case windows forces vs oracle n=4000")
    s = _liquid([(4000, 1.2, 1.0, 21)], "mixed", nvt=200)
    _, obs = _forces(s, 1, 256, energy=True)
    a = s.numpy()
    assert md.md_stats(s.ctx)["staged_fraction"] > 0.5
    na, L = W.n_a_for(4000), W.box_for(4000, 1.2)
    fx, fy, fz, pe, w = O.forces(a["x"], a["y"], a["z"], na, L, "cell")
    num = sum(np.sum((a[k] - f) ** 2) for k, f in zip(("ax", "ay", "az"), (fx, fy, fz)))
    den = sum(np.sum(f ** 2) for f in (fx, fy, fz))
    err = math.sqrt(num / den)
    log(f"  normwise {err:.3e}")
    assert err <= 1e-5
    assert obs[0, 0] == pytest.approx(pe, rel=1e-5)
    assert obs[0, 1] == pytest.approx(w, rel=1e-5)
    s.close()


@pytest.mark.parametrize("rho", [0.02, 2.5e-4])
def test_window_forces_dilute(rho):
    """Dilute boxes: the list builder's coarse candidate test (box 53) and the
    full one (box 229); the few partners per particle span many cells."""
    n = 3000
    log(f"case windows dilute rho={rho}")
    rr = [(n, W.n_a_for(n), W.box_for(n, rho), 1.0, 31)]
    s = md.System(rr, precision="mixed_fixed", init="rsa", min_dist=0.8, skin=0.3)
    ref, _ = _forces(s, 0, 256)
    a, _ = _forces(s, 1, 256)
    for k in ref:
        assert np.array_equal(a[k], ref[k]), k
    s.close()


def _run(prec, windows, wg, steps, graph):
    s = _liquid([(32000, 1.2, 0.5, 41)], prec, nvt=400)
    md.md_set_force_kernel(s.ctx, windows, wg)
    s.build_cells()  # the same rebuild in every variant (a kernel change forces one)
    if graph:
        s.capture(steps // 2)
        s.launch()
        s.launch()
    else:
        s.step_nve(steps)
    s.sync()
    st = md.md_stats(s.ctx)
    out = s.numpy(KEYS)
    assert s.status() == 0
    s.close()
    return out, st


@pytest.mark.parametrize("graph", [False, True])
def test_window_trajectory_equals_direct(graph):
    """N = 32,000 at T = 0.5, 400 NVE steps (several list rebuilds): the
    mixed fixed-point trajectory with windows equals the direct one bit for
    bit, eager and replayed from a graph."""
    log(f"case windows trajectory graph={graph}")
    ref, st0 = _run("mixed_fixed", 0, 256, 400, graph)
    for wg in (256, 64):
        out, st = _run("mixed_fixed", 1, wg, 400, graph)
        log(f"  wg {wg}: rebuilds {st['rebuilds'] - st0['rebuilds']:+.0f} vs direct, "
            f"staged fraction {st['staged_fraction']:.3f}")
        assert st["rebuilds"] == st0["rebuilds"] and st["rebuilds"] >= 2
        for k in KEYS:
            assert np.array_equal(out[k], ref[k]), (wg, k)


def test_window_forces_at_full_size():
    """N = 1,048,576 (the single-system benchmark size): windows equal the
    direct variant bit for bit, and most list parts are staged.  The parts
    left out are mostly those of B wavefronts: 64 B particles spread over
    about five times as many cells as 64 A particles, and the union of their
    stencil rows in the A segment needs more than four windows."""
    wl = W.ka_large()
    r = wl.replicas[0]
    log(f"case windows full size n={r.n}")
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="mixed_fixed", dt=wl.dt,
                  init="lattice", skin=0.4, auto_sync=False)
    s.step_nvt(200, md.NVT_STOCHASTIC, n_reassign=10)
    s.sync()
    ref, _ = _forces(s, 0, 256)
    a, _ = _forces(s, 1, 256)
    st = md.md_stats(s.ctx)
    log(f"  staged fraction {st['staged_fraction']:.3f}, mean list bytes {st['mean_list_bytes']:.1f}")
    assert st["staged_fraction"] > 0.75
    for k in ref:
        assert np.array_equal(a[k], ref[k]), k
    s.close()
