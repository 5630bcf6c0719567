"""Batched contexts against the oracle, replica by replica.

Sixteen replicas of the 256-replica workload (N uniform on [250, 8000],
density 1.2, T evenly on [0.45, 2.0]): the six smallest (boxes below 7.5,
where the list and RDF grids have fewer than three cells per edge) and ten
more of spread sizes.  Every per-replica quantity of the analysis and the
thermostats is compared with the oracle run on that replica alone:

  - pair-distance histograms (Sec. VI.A.1), bit-exact;
  - mean-square displacement against an origin (Eqs. (msdwithi),(msdtw)), 1e-12;
  - one Maxwell-Boltzmann redraw of the stochastic bath (Sec. II.E.1), 1e-12;
  - 20 Nose-Hoover steps (Appendix B): positions 1e-9, xi and ln s 1e-9;
  - 80 FP64 NVE steps of replicas at T = 0.5 and 2.0 (whose lists rebuild on
    different steps): positions, velocities, image counters, 1e-8.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

_CACHE = {}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def chosen():
    wl = W.ka_batch_small()
    reps = list(enumerate(wl.replicas))
    small = sorted(reps, key=lambda t: t[1].n)[:6]
    assert all(r.box < 7.5 for _, r in small)
    rest = sorted((t for t in reps if t not in small and t[1].n <= 4000), key=lambda t: t[1].n)
    pick = small + [rest[k] for k in np.linspace(0, len(rest) - 1, 10).astype(int)]
    return [r for _, r in sorted(pick, key=lambda t: t[0])]


def relaxed_rep(r, T=None):
    """The replica's liquid, relaxed by the oracle's own stochastic bath at T
    (default: the replica's temperature)."""
    T = r.temperature if T is None else T
    key = (r.n, r.seed, T)
    if key not in _CACHE:
        x, y, z = W.lattice_config(r.n, r.box, r.seed, 0.08)
        vx, vy, vz = W.gaussian_velocities(r.n, math.sqrt(T), r.seed + 1)
        st = O.State(x, y, z, vx, vy, vz, r.n_a, r.box)
        st.compute_forces()
        O.run(st, 0.001, 150, nb=5, T=T, seed=r.seed)
        O.run(st, 0.003, 150, nb=10, T=T, seed=r.seed, step0=150)
        _CACHE[key] = (st.x.copy(), st.y.copy(), st.z.copy(), st.vx.copy(), st.vy.copy(), st.vz.copy())
    return _CACHE[key]


def batch(reps, prec="fp64", temps=None):
    pos, vel = [[], [], []], [[], [], []]
    spec = []
    for k, r in enumerate(reps):
        x, y, z, vx, vy, vz = relaxed_rep(r, None if temps is None else temps[k])
        for i, a in enumerate((x, y, z)):
            pos[i].append(a)
        for i, a in enumerate((vx, vy, vz)):
            vel[i].append(a)
        spec.append((r.n, r.n_a, r.box, r.temperature if temps is None else temps[k], r.seed))
    return md.System(spec, precision=prec, positions=[np.concatenate(p) for p in pos],
                     velocities=[np.concatenate(v) for v in vel])


def test_rdf_msd_and_redraw_per_replica():
    reps = chosen()
    log(f"case batch analysis: N = {[r.n for r in reps]}")
    s = batch(reps)
    a0 = s.numpy()
    img0 = s.images()
    # histograms: 200 bins to half the smallest box (one range for every
    # replica), and 25 bins to 2.5 (the finer RDF cell grid in larger boxes)
    lmin = min(r.box for r in reps)
    for dr, nb in ((0.5 * lmin / 200, 200), (0.1, 25)):
        h = s._host(s.rdf(dr, nb)).astype(np.uint64)
        for k, r in enumerate(reps):
            sl = s.replica_slice(k)
            ref = O.rdf_hist(a0["x"][sl], a0["y"][sl], a0["z"][sl], r.n_a, r.box, dr, nb)
            assert np.array_equal(h[k], ref), (k, r.n, dr, np.argwhere(h[k] != ref)[:4])
    # MSD against an origin taken now, after 100 NVE steps
    s.msd_set_origin(3)
    s.step_nve(100)
    got = s.msd(3)
    a = s.numpy()
    img = s.images()
    for k, r in enumerate(reps):
        sl = s.replica_slice(k)
        ux0 = [a0[c][sl] + img0[i][sl] * r.box for i, c in enumerate(("x", "y", "z"))]
        ref = O.msd(a["x"][sl], a["y"][sl], a["z"][sl], img[:, sl], r.n_a, r.box, *ux0)
        assert got[k] == pytest.approx(ref, rel=1e-12), (k, r.n)
    # one redraw of every replica at step 150 (draw tag 150, the replica's
    # index and seed in the counter and key)
    s.step_nvt(50, md.NVT_STOCHASTIC, n_reassign=50)
    a = s.numpy()
    for k, r in enumerate(reps):
        sl = s.replica_slice(k)
        vx, vy, vz = O.mb_velocities(r.n, r.temperature, r.seed, rep=k, tag=150)
        assert np.max(np.abs(a["vx"][sl] - vx)) < 1e-12, (k, r.n)
        assert np.max(np.abs(a["vy"][sl] - vy)) < 1e-12, (k, r.n)
        assert np.max(np.abs(a["vz"][sl] - vz)) < 1e-12, (k, r.n)
    assert s.status() == 0
    s.close()


def test_nose_hoover_per_replica():
    reps = chosen()
    tau = 0.5
    log("case batch nose-hoover")
    s = batch(reps)
    s.step_nvt(20, md.NVT_NOSE_HOOVER, tau=tau)
    a = s.numpy()
    img = s.images()
    th = md.md_thermostat_state(s.ctx, len(reps))
    for k, r in enumerate(reps):
        x, y, z, vx, vy, vz = relaxed_rep(r)
        st = O.State(x, y, z, vx, vy, vz, r.n_a, r.box)
        st.compute_forces()
        O.run_nh(st, 0.005, 20, r.temperature, 3 * r.n * r.temperature * tau ** 2)
        sl = s.replica_slice(k)
        for i, c in enumerate(("x", "y", "z")):
            got = a[c][sl] + img[i][sl] * r.box
            ref = getattr(st, c) + st.img[i] * r.box
            assert np.max(np.abs(got - ref)) < 1e-9, (k, r.n, c)
        assert th[k, 0] == pytest.approx(st.xi, rel=1e-9, abs=1e-12), (k, r.n)
        assert th[k, 1] == pytest.approx(st.lns, rel=1e-9, abs=1e-12), (k, r.n)
    assert s.status() == 0
    s.close()


def test_fp64_trajectories_of_uneven_replicas():
    """Replicas of different size and temperature rebuild their lists on
    different steps; the fused FP64 steps must keep each replica's packed
    positions current whether or not it rebuilt."""
    wl = W.ka_batch_small()
    base = sorted(wl.replicas, key=lambda r: r.n)
    reps = [base[40], base[120], base[200]]
    temps = [0.5, 2.0, 1.0]
    log(f"case fp64 uneven replicas N = {[r.n for r in reps]}")
    s = batch(reps, "fp64", temps)
    s.step_nve(80)
    a = s.numpy()
    img = s.images()
    for k, r in enumerate(reps):
        x, y, z, vx, vy, vz = relaxed_rep(r, temps[k])
        st = O.State(x, y, z, vx, vy, vz, r.n_a, r.box)
        st.compute_forces()
        O.run(st, 0.005, 80)
        sl = s.replica_slice(k)
        for i, c in enumerate(("x", "y", "z")):
            got = a[c][sl] + img[i][sl] * r.box
            ref = getattr(st, c) + st.img[i] * r.box
            assert np.max(np.abs(got - ref)) < 1e-8, (k, r.n, c)
        for c in ("vx", "vy", "vz"):
            assert np.max(np.abs(a[c][sl] - getattr(st, c))) < 1e-8, (k, r.n, c)
        assert np.array_equal(img[:, sl], st.img), (k, r.n)
    st = md.md_stats(s.ctx)
    assert st["rebuilds"] > 0
    assert s.status() == 0
    s.close()
