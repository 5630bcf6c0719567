"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed forms
of the Lennard-Jones pair (Sec. II.B), -grad V by finite differences, Newton's
third law, brute force versus the cell list, an independent pair enumeration
(scipy's periodic k-d tree), scaling laws of the integrator, exact free
flight, time reversibility, the Maxwell-Boltzmann invariants, the Philox
known-answer vectors, the Nose-Hoover conserved quantity (Appendix A) and the
second-order agreement of Eq. (ridotKVLRoman) with Eq. (ridotsolved).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.spatial import cKDTree

import oracle as O
from paper_2001_07089_amd import workload as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAIRS = ("AA", "AB", "BB")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _config(n, rho=1.2, seed=1, jitter=0.12):
    L = W.box_for(n, rho)
    x, y, z = W.lattice_config(n, L, seed, jitter)
    return x, y, z, W.n_a_for(n), L


# ---------------------------------------------------------------- pair model

def test_pair_minimum_and_depth():
    g = _gold("ka_pair_values.json")
    for p, name in enumerate(PAIRS):
        rmin = g["r_min"][name]
        f, v = O.pair_force(p, rmin * rmin)
        assert abs(f) < 1e-12, (name, f)
        # depth -eps shifted by -V(r_c)
        eps = O.KA_EPS[p]
        assert v == pytest.approx(-eps - g["v_rc"][name], rel=1e-12, abs=1e-12)
        # repulsive inside, attractive outside the minimum
        assert O.pair_force(p, (0.95 * rmin) ** 2)[0] > 0
        assert O.pair_force(p, (1.05 * rmin) ** 2)[0] < 0


def test_pair_cutoff_and_shift():
    g = _gold("ka_pair_values.json")
    for p, name in enumerate(PAIRS):
        rc = 2.5 * O.KA_SIGMA[p]
        f, v = O.pair_force(p, rc * rc)
        assert f == 0.0 and v == 0.0  # strict "<" at the cutoff
        f, v = O.pair_force(p, (rc * (1 - 1e-9)) ** 2)
        assert abs(v) < 1e-9  # shifted potential is continuous at r_c
        assert f < 0
        # shift constant: V(r) - V_shifted(r) = V(r_c)
        r = 1.7 * O.KA_SIGMA[p]
        _, vs = O.pair_force(p, r * r)
        eps, s = O.KA_EPS[p], O.KA_SIGMA[p]
        # only the shift is tested here: difference of the shifted values
        r2 = 1.9 * O.KA_SIGMA[p]
        _, vs2 = O.pair_force(p, r2 * r2)
        assert (vs - vs2) == pytest.approx(
            4 * eps * ((s / r) ** 12 - (s / r) ** 6) - 4 * eps * ((s / r2) ** 12 - (s / r2) ** 6),
            rel=1e-12)
        assert vs == pytest.approx(4 * eps * ((s / r) ** 12 - (s / r) ** 6) - g["v_rc"][name],
                                   rel=1e-11)


def test_pair_golden_values():
    g = _gold("ka_pair_values.json")
    f, v = O.pair_force(0, 0.64)
    assert f * 0.8 == pytest.approx(g["f_times_r_AA_at_0.8"], rel=1e-11)
    assert v == pytest.approx(g["v_unshifted_AA_at_0.8"] - g["v_rc"]["AA"], rel=1e-11)


def test_pair_force_is_minus_dv_dr():
    for p in range(3):
        for r in np.linspace(0.75, 2.4, 23) * O.KA_SIGMA[p]:
            h = 1e-6 * r
            _, vp = O.pair_force(p, (r + h) ** 2)
            _, vm = O.pair_force(p, (r - h) ** 2)
            f, _ = O.pair_force(p, r * r)
            assert f * r == pytest.approx(-(vp - vm) / (2 * h), rel=1e-7, abs=1e-9)


def test_pair_types_by_index_block():
    # two particles at the AB minimum: only the AB pair sits at zero force
    L = 10.0
    rmin = 0.8 * 2 ** (1 / 6)
    x = np.array([1.0, 1.0 + rmin]); y = np.ones(2); z = np.ones(2)
    fx, fy, fz, pe, w = O.forces(x, y, z, 1, L, "brute")
    assert abs(fx[0]) < 1e-12 and pe == pytest.approx(-1.5 + 0.024475336704, rel=1e-11)
    fx, _, _, pe, _ = O.forces(x, y, z, 2, L, "brute")  # both A: AA pair, repulsive
    assert fx[0] < 0 < fx[1]
    fx, _, _, pe, _ = O.forces(x, y, z, 0, L, "brute")  # both B
    assert fx[0] < 0 < fx[1]


# ---------------------------------------------------------- force field sums

def test_forces_minus_gradient_fd():
    n = 60
    x, y, z, na, L = _config(n, rho=0.9, seed=3)
    fx, fy, fz, pe, _ = O.forces(x, y, z, na, L, "brute")
    rng = np.random.default_rng(0)
    h = 1e-6
    for i in rng.choice(n, 8, replace=False):
        for arr, f in ((x, fx), (y, fy), (z, fz)):
            old = arr[i]
            arr[i] = old + h
            pp = O.forces(x, y, z, na, L, "brute")[3]
            arr[i] = old - h
            pm = O.forces(x, y, z, na, L, "brute")[3]
            arr[i] = old
            assert f[i] == pytest.approx(-(pp - pm) / (2 * h), rel=1e-6, abs=1e-6)


def test_newton_third_law():
    x, y, z, na, L = _config(500, seed=5)
    for method in ("brute", "cell"):
        fx, fy, fz, _, _ = O.forces(x, y, z, na, L, method)
        scale = np.abs(fx).sum() + np.abs(fy).sum() + np.abs(fz).sum()
        for f in (fx, fy, fz):
            assert abs(f.sum()) <= 1e-12 * scale


@pytest.mark.parametrize("n,rho,seed", [(500, 1.2, 1), (864, 1.2, 2), (3000, 1.1, 3), (2000, 1.3, 4)])
def test_brute_equals_cell(n, rho, seed):
    x, y, z, na, L = _config(n, rho, seed)
    b = O.forces(x, y, z, na, L, "brute")
    c = O.forces(x, y, z, na, L, "cell")
    for k in range(3):
        assert np.max(np.abs(b[k] - c[k])) <= 1e-12 * max(1.0, np.max(np.abs(b[k])))
    assert c[3] == pytest.approx(b[3], rel=1e-12)
    assert c[4] == pytest.approx(b[4], rel=1e-12)


def test_pair_enumeration_matches_kdtree():
    """PE and virial re-summed over pairs found by scipy's periodic k-d tree."""
    x, y, z, na, L = _config(700, seed=7)
    fx, fy, fz, pe, w = O.forces(x, y, z, na, L, "cell")
    pos = np.stack([x, y, z], axis=1)
    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(2.5, output_type="ndarray")
    pe2 = 0.0
    w2 = 0.0
    cnt = 0
    for i, j in pairs:
        p = int(i >= na) + int(j >= na)
        d = pos[i] - pos[j]
        d -= L * np.round(d / L)
        r2 = float(d @ d)
        f, v = O.pair_force(p, r2)
        pe2 += v
        w2 += f * r2
        cnt += int(r2 < (2.5 * O.KA_SIGMA[p]) ** 2)
    assert pe == pytest.approx(pe2, rel=1e-11)
    assert w == pytest.approx(w2, rel=1e-11)
    assert cnt > 20 * 700 // 2


def test_translation_invariance():
    x, y, z, na, L = _config(800, seed=8)
    f0 = O.forces(x, y, z, na, L, "cell")
    sh = np.array([3.3, -7.1, 0.4 * L])
    xs = np.mod(x + sh[0], L); ys = np.mod(y + sh[1], L); zs = np.mod(z + sh[2], L)
    xs[xs >= L] = 0; ys[ys >= L] = 0; zs[zs >= L] = 0
    f1 = O.forces(xs, ys, zs, na, L, "cell")
    for k in range(3):
        assert np.max(np.abs(f1[k] - f0[k])) < 1e-9
    assert f1[3] == pytest.approx(f0[3], rel=1e-11)


def test_virial_is_volume_derivative():
    x, y, z, na, L = _config(400, rho=1.1, seed=9)
    _, _, _, _, w = O.forces(x, y, z, na, L, "brute")
    h = 1e-6

    def U(lam):
        return O.forces(x * lam, y * lam, z * lam, na, L * lam, "brute")[3]
    dU = (U(1 + h) - U(1 - h)) / (2 * h)
    assert w == pytest.approx(-dU, rel=1e-6)


def test_min_distance_matches_kdtree():
    x, y, z, na, L = _config(600, seed=10)
    d = O.min_distance(x, y, z, L)
    tree = cKDTree(np.stack([x, y, z], 1), boxsize=L)
    dd, _ = tree.query(np.stack([x, y, z], 1), k=2)
    assert d == pytest.approx(dd[:, 1].min(), rel=1e-12)


# ------------------------------------------------------------- integrators

_LIQ = {}


def _liquid(n=500, T=1.0, seed=11):
    """A relaxed liquid at temperature T: jittered lattice, then stochastic-bath
    steps (Sec. III.G) with a small step until the lattice overlap energy is gone."""
    key = (n, T, seed)
    if key not in _LIQ:
        x, y, z, na, L = _config(n, seed=seed, jitter=0.08)
        vx, vy, vz = W.gaussian_velocities(n, math.sqrt(T), seed + 1)
        st = O.State(x, y, z, vx, vy, vz, na, L)
        st.compute_forces()
        O.run(st, 0.001, 200, nb=5, T=T, seed=seed)
        O.run(st, 0.003, 300, nb=10, T=T, seed=seed, step0=200)
        _LIQ[key] = st
    return _LIQ[key].copy()


def test_free_flight_is_exact():
    m = O.model(eps=(0.0, 0.0, 0.0))
    st = _liquid()
    st.compute_forces(m=m)
    x0 = O.unwrapped(st.x, st.y, st.z, st.img, st.L)
    v0 = (st.vx.copy(), st.vy.copy(), st.vz.copy())
    dt, nsteps = 0.01, 700  # long enough to cross the box many times
    O.run(st, dt, nsteps, m=m)
    xu = O.unwrapped(st.x, st.y, st.z, st.img, st.L)
    t = dt * nsteps
    for k in range(3):
        assert np.max(np.abs(xu[k] - (x0[k] + v0[k] * t))) < 1e-9
    msd = O.msd(st.x, st.y, st.z, st.img, st.na, st.L, *x0)
    v2 = v0[0] ** 2 + v0[1] ** 2 + v0[2] ** 2
    assert msd[0] == pytest.approx(v2[:st.na].mean() * t * t, rel=1e-10)
    assert msd[1] == pytest.approx(v2[st.na:].mean() * t * t, rel=1e-10)
    assert np.all(st.x >= 0) and np.all(st.x < st.L)
    assert np.abs(st.img).max() > 2


def test_nve_energy_error_scales_as_dt_squared():
    base = _liquid(n=500, T=0.8, seed=12)
    O.run(base, 0.002, 200)  # relax the jittered start
    base.vx, base.vy, base.vz = O.mb_velocities(base.n, 0.8, 7)
    base.compute_forces()
    amps = []
    T_phys = 0.5
    for dt in (0.004, 0.002, 0.001):
        st = base.copy()
        e = O.run(st, dt, int(round(T_phys / dt)))
        et = e[:, 0] + e[:, 1]
        amps.append(et.max() - et.min())
    r1, r2 = amps[0] / amps[1], amps[1] / amps[2]
    assert 2.8 < r1 < 5.5 and 2.8 < r2 < 5.5, amps


def test_nve_time_reversible():
    st = _liquid(n=300, T=0.6, seed=13)
    s0 = st.copy()
    O.run(st, 0.003, 40)
    st.vx *= -1; st.vy *= -1; st.vz *= -1
    O.run(st, 0.003, 40)
    a = O.unwrapped(st.x, st.y, st.z, st.img, st.L)
    b = O.unwrapped(s0.x, s0.y, s0.z, s0.img, s0.L)
    for k in range(3):
        assert np.max(np.abs(a[k] - b[k])) < 1e-8
    assert np.max(np.abs(st.vx + s0.vx)) < 1e-7


def test_nve_conserves_energy_and_momentum():
    st = _liquid(n=864, T=1.0, seed=14)
    O.run(st, 0.002, 200)
    p0 = np.array([st.vx.sum(), st.vy.sum(), st.vz.sum()])
    e = O.run(st, 0.005, 400)
    et = e[:, 0] + e[:, 1]
    assert abs(et[-1] - et[0]) / abs(et[0]) < 2e-4
    p1 = np.array([st.vx.sum(), st.vy.sum(), st.vz.sum()])
    assert np.max(np.abs(p1 - p0)) < 1e-9


def test_brute_and_cell_trajectories_agree_short():
    st1 = _liquid(n=700, T=1.0, seed=15)
    st2 = st1.copy()
    O.run(st1, 0.005, 20, method="brute")
    O.run(st2, 0.005, 20, method="cell")
    assert np.max(np.abs(st1.x - st2.x)) < 1e-9


# ----------------------------------------------------------- thermostats

def test_philox_known_answers():
    for v in _gold("philox4x32_10_kat.json")["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        out = [int(h, 16) for h in v["out"]]
        assert O.philox4x32_10(ctr, key).tolist() == out


def test_gaussians_are_standard_normal():
    g = np.array([O.gauss3(12345, 3, 7, i) for i in range(20000)]).ravel()
    assert abs(g.mean()) < 4 / math.sqrt(g.size)
    assert abs(g.var() - 1) < 4 * math.sqrt(2 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # components are uncorrelated
    gg = g.reshape(-1, 3)
    c = np.corrcoef(gg.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.05


def test_mb_flow_chart_invariants():
    n, T = 1000, 0.2
    vx, vy, vz = O.mb_velocities(n, T, seed=99, rep=2, tag=5)
    for v in (vx, vy, vz):
        assert abs(v.sum()) < 1e-12
    assert (vx @ vx + vy @ vy + vz @ vz) == pytest.approx(3 * n * T, rel=1e-13)
    # a different tag or replica gives a different draw
    wx, _, _ = O.mb_velocities(n, T, seed=99, rep=2, tag=6)
    assert np.max(np.abs(wx - vx)) > 0.1


def test_mb_draw_of_one_and_two_particles():
    """Two particles: after the centre-of-mass step their velocities are equal
    and opposite, and the rescale still gives sum v^2 = 3 N T.  One particle:
    nothing is left after that step, and it stays at rest (no 0/0)."""
    vx, vy, vz = O.mb_velocities(2, 0.7, seed=5, rep=0, tag=1)
    for v in (vx, vy, vz):
        assert v[0] == pytest.approx(-v[1], rel=1e-14, abs=1e-15)
    assert (vx @ vx + vy @ vy + vz @ vz) == pytest.approx(3 * 2 * 0.7, rel=1e-13)
    vx, vy, vz = O.mb_velocities(1, 0.7, seed=5, rep=0, tag=1)
    assert vx.tolist() == [0.0] and vy.tolist() == [0.0] and vz.tolist() == [0.0]


def test_stochastic_bath_resets_temperature():
    st = _liquid(n=500, T=1.5, seed=16)
    e = O.run(st, 0.005, 50, nb=10, T=0.2, seed=3)
    n = st.n
    for s in range(10, 51, 10):
        ke = e[s - 1, 0]
        assert 2 * ke / (3 * n) == pytest.approx(0.2, rel=1e-13)


def test_nose_hoover_conserves_extended_energy():
    st = _liquid(n=500, T=1.0, seed=17)
    O.run(st, 0.002, 200)
    T, dt = 0.7, 0.001
    Q = 3 * st.n * T * (100 * 0.005) ** 2
    e = O.run_nh(st, dt, 600, T, Q)
    H = np.array([O.nh_conserved(r, st.n, T, Q) for r in e])
    # H~ of Eq. (HNosetilde) stays put (its residual drift is the O(dt^2)
    # integration error checked by the next test) while the friction switches
    # on to cool the hotter-than-bath system
    assert np.max(np.abs(H - H[0])) < 1e-4 * abs(H[0])
    assert e[:, 3].max() > 0.3
    assert 2 * e[-1, 0] / (3 * st.n) < 0.95


def test_nose_hoover_drift_scales_with_dt():
    st0 = _liquid(n=400, T=1.0, seed=18)
    O.run(st0, 0.002, 200)
    T = 0.7
    Q = 3 * st0.n * T * 0.5 ** 2
    amps = []
    for dt in (0.002, 0.001):
        st = st0.copy()
        e = O.run_nh(st, dt, int(round(0.6 / dt)), T, Q)
        H = np.array([O.nh_conserved(r, st.n, T, Q) for r in e])
        amps.append(H.max() - H.min())
    assert 3.0 < amps[0] / amps[1] < 5.0, amps


def test_nose_hoover_velocity_forms_agree_to_third_order():
    st0 = _liquid(n=300, T=1.0, seed=19)
    O.run(st0, 0.002, 100)
    T = 0.5
    Q = 3 * st0.n * T * 1.0 ** 2  # heavy bath: xi_a stays close to the large xi
    st0.xi = 3.0
    devs = []
    for dt in (0.01, 0.005, 0.0025):
        a = st0.copy(); b = st0.copy()
        O.run_nh(a, dt, 1, T, Q, exact_solve=False)
        O.run_nh(b, dt, 1, T, Q, exact_solve=True)
        devs.append(np.max(np.abs(a.vx - b.vx)))
    assert 6.0 < devs[0] / devs[1] < 10.0 and 6.0 < devs[1] / devs[2] < 10.0, devs


# ----------------------------------------------------------------- analysis

def test_rdf_counts_match_kdtree():
    x, y, z, na, L = _config(800, seed=20, jitter=0.3)
    dr, nbins = 0.1, int(L / 2 / 0.1)
    h = O.rdf_hist(x, y, z, na, L, dr, nbins)
    pos = np.stack([x, y, z], 1)
    tree = cKDTree(pos, boxsize=L)
    typ = (np.arange(x.size) >= na).astype(int)
    cum = np.zeros((3, nbins + 1), np.int64)
    for b in range(1, nbins + 1):
        pr = tree.query_pairs(b * dr * (1 - 1e-14), output_type="ndarray")
        p = typ[pr[:, 0]] + typ[pr[:, 1]]
        for k in range(3):
            cum[k, b] = np.count_nonzero(p == k)
    counts = np.diff(cum, axis=1)
    counts[0] *= 2
    counts[2] *= 2
    assert np.array_equal(counts.astype(np.uint64), h)


def test_rdf_uniform_positions_is_one():
    n, L = 400, 7.0
    na = W.n_a_for(n)
    dr = 0.25
    nbins = int(L / 2 / dr)
    h = np.zeros((3, nbins), np.uint64)
    nmeas = 60
    for s in range(nmeas):
        x, y, z = W.uniform_config(n, L, 1000 + s)
        O.rdf_hist(x, y, z, na, L, dr, nbins, h)
    r, g = O.rdf_normalize(h, n, na, L, dr, nmeas)
    sel = r > 1.0
    for k in range(3):
        gk = g[k, sel]
        # expected 1 in every bin; pooled mean within a few percent
        assert abs(gk.mean() - 1.0) < 0.03, (k, gk.mean())
        chi = ((h[k, sel].astype(float) / (gk / 1.0 + 1e-300)) > 0).all()
        assert chi


def test_rdf_liquid_excludes_core():
    st = _liquid(n=864, T=1.0, seed=21)
    O.run(st, 0.004, 300)
    h = O.rdf_hist(st.x, st.y, st.z, st.na, st.L, 0.05, int(st.L / 2 / 0.05))
    assert h[0, :14].sum() == 0  # g_AA = 0 below 0.7 sigma
    assert h[1, :12].sum() == 0


def test_msd_hand_case():
    n, na, L = 10, 6, 5.0
    x = np.full(n, 4.5); y = np.full(n, 1.0); z = np.full(n, 1.0)
    img = np.zeros((3, n), np.int32)
    x0u, y0u, z0u = O.unwrapped(x, y, z, img, L)
    # A particles cross the +x face: position 0.5 in the next image (moved by 1)
    x2 = x.copy(); img2 = img.copy()
    x2[:na] = 0.5; img2[0, :na] = 1
    out = O.msd(x2, y, z, img2, na, L, x0u, y0u, z0u)
    assert out[0] == pytest.approx(1.0, rel=1e-15) and out[1] == 0.0


def test_log_schedule_closed_form():
    for nmd, t0, kmax in ((1000, 1.0, 60), (10000, 1.0, 60), (5000, 10.0, 40)):
        s = O.log_schedule(nmd, t0, kmax)
        A = (nmd / t0) ** (1.0 / kmax)
        ref = sorted({int(round(t0 * A ** k)) for k in range(kmax + 1)})
        ref = [v for v in ref if 1 <= v <= nmd]
        assert s.tolist() == ref
        assert s[-1] == nmd
    s = O.log_schedule(1000, 1.0, 60)
    assert len(s) == 50 and s[:11].tolist() == list(range(1, 12))


def test_van_hove_self_closed_form():
    """Self van Hove histogram: A particles displaced by one common vector all
    land in the bin of its length, B particles by another; a displacement that
    crosses the box several times counts through the image counters; lengths
    at or past n_bins * dr are not counted."""
    n, na, L = 50, 40, 6.0
    rng = np.random.default_rng(3)
    x0, y0, z0 = (rng.uniform(0, L, n) for _ in range(3))
    img0 = np.zeros((3, n), np.int32)
    ux0, uy0, uz0 = O.unwrapped(x0, y0, z0, img0, L)
    shA, shB = np.array([0.31, -0.4, 1.2]), np.array([2.0 * L + 0.52, 0.0, 0.0])  # lengths off bin edges
    shift = np.where(np.arange(n)[None, :] < na, shA[:, None], shB[:, None])
    u = np.array([x0, y0, z0]) + shift
    img = np.floor(u / L).astype(np.int32)
    w = u - img * L
    dr = 0.05
    h = O.van_hove_self(w[0], w[1], w[2], img, na, L, ux0, uy0, uz0, dr, 400)
    binA, binB = int(np.linalg.norm(shA) / dr), int(np.linalg.norm(shB) / dr)
    assert h[0, binA] == na and h[0].sum() == na
    assert h[1, binB] == n - na and h[1].sum() == n - na
    h2 = O.van_hove_self(w[0], w[1], w[2], img, na, L, ux0, uy0, uz0, dr, binB)  # B beyond the range
    assert h2[1].sum() == 0 and h2[0].sum() == na
    # MSD of the same configuration is the squared common length per species
    m = O.msd(w[0], w[1], w[2], img, na, L, ux0, uy0, uz0)
    assert m[0] == pytest.approx(shA @ shA, rel=1e-12) and m[1] == pytest.approx(shB @ shB, rel=1e-12)


_PLANAR = {}


def _planar_liquid(n=400, seed=7, T=0.6):
    """Planar 65:35 KA system at N/L^2 = 1.204 (appendix exercise), z = vz = 0,
    relaxed with the planar bath (a copy of a cached state)."""
    key = (n, seed, T)
    if key not in _PLANAR:
        _PLANAR[key] = _make_planar(n, seed, T)
    st = _PLANAR[key]
    c = O.State(st.x, st.y, st.z, st.vx, st.vy, st.vz, st.na, st.L)
    c.compute_forces("brute")
    return c


def _make_planar(n, seed, T):
    L = math.sqrt(n / 1.204)
    na = int(round(0.65 * n))
    m = int(math.ceil(math.sqrt(n)))
    a = L / m
    rng = np.random.default_rng(seed)
    sites = rng.permutation(m * m)[:n]
    x = (sites % m + 0.5 + rng.uniform(-0.05, 0.05, n)) * a
    y = (sites // m + 0.5 + rng.uniform(-0.05, 0.05, n)) * a
    z = np.zeros(n)
    vx, vy, vz = O.mb_velocities(n, T, 99, dim=2)
    st = O.State(x % L, y % L, z, vx, vy, vz, na, L)
    st.compute_forces("brute")
    O.run(st, 0.00025, 300, method="brute", nb=5, T=T, seed=99, dim=2)
    O.run(st, 0.002, 3000, method="brute", nb=10, T=T, seed=99, dim=2, step0=300)
    return st


def test_planar_maxwell_boltzmann_draw():
    """Planar flow chart: vz = 0, zero momentum, sum v^2 = 2 N T exactly, and
    (x, y) are the three-dimensional draw's first two Gaussians recentred and
    rescaled (one common factor)."""
    n, T = 500, 0.7
    vx2, vy2, vz2 = O.mb_velocities(n, T, 11, rep=3, tag=20, dim=2)
    vx3, vy3, _ = O.mb_velocities(n, T, 11, rep=3, tag=20)
    assert np.all(vz2 == 0.0)
    assert abs(vx2.sum()) < 1e-12 and abs(vy2.sum()) < 1e-12
    assert np.sum(vx2 ** 2 + vy2 ** 2) == pytest.approx(2 * n * T, rel=1e-13)
    ratio = vx2 / vx3
    assert np.allclose(ratio, ratio[0], rtol=1e-12) and np.allclose(vy2 / vy3, ratio[0], rtol=1e-12)


def test_planar_system_stays_planar_and_conserves_energy():
    st = _planar_liquid()
    assert np.all(st.z == 0.0) and np.all(st.vz == 0.0) and np.all(st.az == 0.0)
    e = O.run(st, 0.001, 300, method="brute")
    tot = e[:, 0] + e[:, 1]
    assert np.all(st.z == 0.0) and np.all(st.img[2] == 0)
    assert np.max(np.abs(tot - tot[0])) / abs(tot[0]) < 1e-4


def test_planar_nose_hoover_conserves_with_2n_degrees():
    """Planar Nose-Hoover: the extended energy with X = 2N is conserved; with
    X = 3N (the three-dimensional count) it drifts, so the oracle's X follows
    the dimension."""
    st = _planar_liquid()
    n, T, tau = st.n, 0.4, 0.2
    Q = 2 * n * T * tau ** 2
    e = O.run_nh(st, 0.001, 400, T, Q, method="brute", dim=2)
    h2 = np.array([O.nh_conserved(r, n, T, Q, dim=2) for r in e])
    h3 = np.array([O.nh_conserved(r, n, T, Q, dim=3) for r in e])
    d2 = np.max(np.abs(h2 - h2[0])) / abs(h2[0])
    d3 = np.max(np.abs(h3 - h3[0])) / abs(h3[0])
    assert d2 < 2e-4 and d3 > 100 * d2


def test_planar_square_lattice_rdf():
    """Pair histogram of a perfect square lattice (all A): the neighbour
    shells of the square lattice per particle (AA counts 2 per pair, so a
    shell of k neighbours holds k N counts); the planar normalisation turns
    the first shell into a coordination number of exactly 4."""
    m = 20
    a = 1.13  # a, a*sqrt(2), 2a all lie well inside their bins of width 0.05
    L = m * a
    n = m * m
    i = np.arange(n)
    x, y, z = (i % m + 0.5) * a, (i // m + 0.5) * a, np.zeros(n)
    dr = 0.05
    h = O.rdf_hist(x, y, z, n, L, dr, 60)
    # within r_max = 3.0: 4 at a, 4 at a*sqrt(2), 4 at 2a, 8 at a*sqrt(5)
    for r, k in ((a, 4), (a * math.sqrt(2), 4), (2 * a, 4), (a * math.sqrt(5), 8)):
        assert h[0, int(r / dr)] == k * n
    assert int(h[0].sum()) == 20 * n
    rmid, g = O.rdf_normalize(h, n, n, L, dr, 1, dim=2)
    rho = n / L ** 2
    b = int(a / dr)
    shell = math.pi * (((b + 1) * dr) ** 2 - (b * dr) ** 2)
    assert rho * g[0, b] * shell * (n - 1) / n == pytest.approx(4.0, rel=1e-12)


# ---------------------------------------------- LAMMPS conventions (Sec. IV.B, VI.A.3)

def test_pe_lj_cut_pair_closed_forms():
    """Two particles, one pair type at a time, placed across the periodic
    boundary: Eq. (VKALJ) without the shift inside r_c, zero beyond."""
    L = 10.0
    for p, na in ((0, 2), (1, 1), (2, 0)):
        eps, sig = O.KA_EPS[p], O.KA_SIGMA[p]
        for r in (0.93 * sig, 1.31 * sig, 2.37 * sig, 2.61 * sig):
            x = np.array([0.2, (0.2 - r) % L])
            y = np.array([3.0, 3.0])
            z = np.array([9.9, 9.9])
            want = 4.0 * eps * ((sig / r) ** 12 - (sig / r) ** 6) if r < 2.5 * sig else 0.0
            assert O.pe_lj_cut(x, y, z, na, L) == pytest.approx(want, rel=1e-12, abs=1e-14), (p, r)


def test_pe_lj_cut_exceeds_the_shifted_energy_by_one_shift_per_pair():
    """Unshifted minus shifted energy = sum over pairs inside r_c(ab) of
    V_ab(r_c) = 4 eps_ab (0.4^12 - 0.4^6); pairs counted with a periodic k-d tree."""
    x, y, z, na, L = _config(600, seed=5, jitter=0.2)
    _, _, _, pe_shifted, _ = O.forces(x, y, z, na, L, "brute")
    pe_cut = O.pe_lj_cut(x, y, z, na, L)
    pts = np.mod(np.stack([x, y, z], axis=1), L)
    pairs = cKDTree(pts, boxsize=L).query_pairs(2.5 * max(O.KA_SIGMA), output_type="ndarray")
    d = pts[pairs[:, 0]] - pts[pairs[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt(np.sum(d * d, axis=1))
    p = (pairs[:, 0] >= na).astype(int) + (pairs[:, 1] >= na).astype(int)
    sig = np.array(O.KA_SIGMA)[p]
    inside = r < 2.5 * sig
    shift = np.array([4.0 * e * (0.4 ** 12 - 0.4 ** 6) for e in O.KA_EPS])
    want = float(np.sum(shift[p[inside]]))
    assert np.count_nonzero(inside) > 1000
    assert pe_cut - pe_shifted == pytest.approx(want, rel=1e-9)


def test_lammps_rdf_coordination_numbers_of_a_simple_cubic_lattice():
    """All-A simple cubic lattice: the coordination number c_AA steps through
    the lattice shells 6 (a), 12 (a sqrt 2), 8 (a sqrt 3), 6 (2a), 24 (a sqrt 5),
    i.e. 6, 18, 26, 32, 56, at the bins holding those radii; the g column
    integrates back to c."""
    m, a = 8, 1.07
    L = m * a
    n = m ** 3
    i = np.arange(n)
    x, y, z = (i % m + 0.5) * a, ((i // m) % m + 0.5) * a, (i // (m * m) + 0.5) * a
    rcut, nbins = 2.5, 25
    dr = rcut / nbins
    h = O.rdf_hist(x, y, z, n, L, dr, nbins)
    t = O.lammps_rdf_table(h, n, n, L, rcut, nbins)
    prev = 0
    for r, c in ((a, 6), (a * math.sqrt(2), 18), (a * math.sqrt(3), 26), (2 * a, 32), (a * math.sqrt(5), 56)):
        b = int(r / dr)
        assert t[b, 3] == pytest.approx(c, rel=1e-12)
        assert t[b - 1, 3] == pytest.approx(prev, abs=1e-12)
        prev = c
    assert t[-1, 3] == pytest.approx(56, rel=1e-12)
    shell = (4.0 * math.pi / 3.0) * ((t[:, 0] * dr) ** 3 - ((t[:, 0] - 1) * dr) ** 3)
    assert np.sum(t[:, 2] * shell) * (n - 1) / L ** 3 == pytest.approx(56, rel=1e-12)
    assert np.all(t[:, 4:] == 0.0)  # no B particles
