"""Degenerate and ragged inputs through the C ABI against the FP64 oracle:
replicas with one species only (no B, or no A particles), replicas of one and
two particles, and a batch that mixes them with an ordinary liquid.  Every
segment of a replica is padded to a whole wavefront, so these exercise empty
segments, wavefronts with a single real lane, and lists with no partners."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5, "mixed_fixed": 1e-5}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(a, b):
    num = sum(np.sum((a[k] - b[k]) ** 2) for k in range(3))
    den = sum(np.sum(b[k] ** 2) for k in range(3))
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def liquid(n, na, seed, rho=1.2):
    L = W.box_for(n, rho)
    x, y, z = W.lattice_config(n, L, seed, 0.08)
    return (x, y, z), L


def build(specs, precision, **kw):
    """specs: list of (positions (x, y, z), velocities (vx, vy, vz), n_a, L, T)."""
    reps, pos, vel = [], [[], [], []], [[], [], []]
    for i, (p, v, na, L, T) in enumerate(specs):
        reps.append((p[0].size, na, L, T, 300 + i))
        for k in range(3):
            pos[k].append(np.asarray(p[k], np.float64))
            vel[k].append(np.asarray(v[k], np.float64))
    return md.System(reps, precision=precision, positions=[np.concatenate(a) for a in pos],
                     velocities=[np.concatenate(a) for a in vel], **kw)


def check_forces(s, specs, prec):
    """GPU forces of every replica against the oracle at the GPU's positions."""
    a = s.numpy()
    off = 0
    for (p, _, na, L, _) in specs:
        n = p[0].size
        sl = slice(off, off + n)
        fx, fy, fz, _, _ = O.forces(a["x"][sl], a["y"][sl], a["z"][sl], na, L, "brute")
        err = normwise((a["ax"][sl], a["ay"][sl], a["az"][sl]), (fx, fy, fz))
        assert err <= TOL[prec], (prec, n, na, err)
        off += n


@pytest.mark.parametrize("prec", ["fp64", "mixed_fixed"])
@pytest.mark.parametrize("species", ["A", "B"])
def test_one_species_replica(prec, species):
    """n_a = n (a one-component LJ liquid of A particles) or n_a = 0 (of B
    particles): the other segment is empty.  Forces at the start and after 50
    NVE steps (the lists are reused and rebuilt in between)."""
    n = 500
    na = n if species == "A" else 0
    log(f"case one species {species} {prec}")
    p, L = liquid(n, na, 11)
    v = W.gaussian_velocities(n, 1.0, 12)
    specs = [(p, v, na, L, 1.0)]
    s = build(specs, prec)
    check_forces(s, specs, prec)
    s.step_nve(50)
    assert s.status() == 0
    check_forces(s, specs, prec)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_fixed"])
def test_one_and_two_particle_replicas(prec):
    """A lone particle feels no force and flies freely; a pair at r = 1.1
    feels the pair force of its types (AA, AB or BB by n_a)."""
    log(f"case tiny replicas {prec}")
    L = 6.0  # L/2 above the largest cutoff, r_c,AA = 2.5
    z1 = (np.array([1.5]), np.array([2.0]), np.array([2.5]))
    v1 = (np.array([0.3]), np.array([-0.2]), np.array([0.1]))
    p2 = (np.array([1.0, 2.1]), np.array([1.0, 1.0]), np.array([1.0, 1.0]))
    v0 = (np.zeros(2), np.zeros(2), np.zeros(2))
    specs = [(z1, v1, 1, L, 1.0), (p2, v0, 2, L, 1.0), (p2, v0, 1, L, 1.0), (p2, v0, 0, L, 1.0)]
    s = build(specs, prec)
    a = s.numpy()
    assert a["ax"][0] == 0.0 and a["ay"][0] == 0.0 and a["az"][0] == 0.0
    check_forces(s, specs, prec)
    for r, p in enumerate((0, 1, 2)):  # pair types AA, AB, BB
        fx = a["ax"][1 + 2 * r]
        f, _ = O.pair_force(p, 1.1 ** 2)  # F_i = f (r_i - r_j); x_i - x_j = -1.1 for the left one
        assert fx == pytest.approx(-1.1 * f, rel=TOL[prec] * 10), (p, fx, f)
        assert a["ax"][2 + 2 * r] == pytest.approx(-fx, rel=1e-12)
    s.step_nve(10)
    assert s.status() == 0
    a = s.numpy()
    dt = s.cfg.dt
    assert a["x"][0] == pytest.approx(1.5 + 10 * dt * 0.3, rel=1e-12)
    assert a["vx"][0] == pytest.approx(0.3, rel=1e-12)
    s.close()


def test_lone_particle_under_the_stochastic_bath_stays_at_rest():
    """The velocity redraw subtracts the centre-of-mass velocity, which for a
    single particle is all of it: the redraw leaves it at rest (no 0/0), as
    the oracle's flow chart does."""
    log("case lone particle bath")
    L = 6.0
    p = (np.array([1.5]), np.array([2.0]), np.array([2.5]))
    v = (np.array([0.3]), np.array([-0.2]), np.array([0.1]))
    s = build([(p, v, 1, L, 1.0)], "mixed_fixed")
    s.step_nvt(10, md.NVT_STOCHASTIC, n_reassign=5)
    assert s.status() == 0
    a = s.numpy()
    assert a["vx"][0] == 0.0 and a["vy"][0] == 0.0 and a["vz"][0] == 0.0
    assert np.isfinite(a["x"][0])
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fixed"])
def test_batch_mixing_degenerate_and_ordinary_replicas(prec):
    """One context holding a lone particle, a pair, a one-species B liquid and
    an ordinary 80:20 liquid: per-replica forces before and after 40 NVE
    steps, and the lone particle's free flight."""
    log(f"case mixed batch {prec}")
    L6 = 6.0
    z1 = (np.array([1.5]), np.array([2.0]), np.array([2.5]))
    v1 = (np.array([0.3]), np.array([-0.2]), np.array([0.1]))
    p2 = (np.array([1.0, 2.1]), np.array([1.0, 1.0]), np.array([1.0, 1.0]))
    v2 = (np.array([0.1, -0.1]), np.zeros(2), np.zeros(2))
    pb, Lb = liquid(300, 0, 21)
    vb = W.gaussian_velocities(300, 0.8, 22)
    pm, Lm = liquid(700, W.n_a_for(700), 23)
    vm = W.gaussian_velocities(700, 0.8, 24)
    specs = [(z1, v1, 1, L6, 1.0), (p2, v2, 1, L6, 1.0), (pb, vb, 0, Lb, 0.8), (pm, vm, W.n_a_for(700), Lm, 0.8)]
    s = build(specs, prec)
    check_forces(s, specs, prec)
    s.step_nve(40)
    assert s.status() == 0
    check_forces(s, specs, prec)
    a = s.numpy()
    assert a["x"][0] == pytest.approx(1.5 + 40 * s.cfg.dt * 0.3, rel=1e-12)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fixed"])
def test_runaway_pair_sets_its_bit(prec):
    """Two A particles 0.5 apart, as a random start can leave them (Sec. II.F):
    the repulsion throws them apart by several sigma in the first step, far
    more than half the smallest sigma, which sets KAMD_DEV_RUNAWAY and
    nothing else; a pair at r = 1.1 moves a tiny fraction of it and sets
    nothing."""
    L = 6.0
    v0 = (np.zeros(2), np.zeros(2), np.zeros(2))
    for r, expect in ((0.5, True), (1.1, False)):
        log(f"case runaway {prec} r={r}")
        p = (np.array([2.0, 2.0 + r]), np.array([3.0, 3.0]), np.array([3.0, 3.0]))
        s = build([(p, v0, 2, L, 1.0)], prec)
        assert s.status() == 0
        s.step_nve(1)
        w = s.status()
        assert w == (md.DEV_RUNAWAY if expect else 0), (r, w)
        # the pair has flown apart (beyond the cutoff): stopped, and with the
        # word cleared, later steps are ordinary
        s.scale_velocities([0.0])
        s.clear_status()
        s.step_nve(5)
        assert s.status() == 0
        s.close()
