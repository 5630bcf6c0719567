"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Inputs are seeded synthetic Kob-Andersen liquids (jittered lattice relaxed by
the oracle's own stochastic-bath run) fed identically to both sides.
Tolerances: forces normwise 1e-12 (FP64) / 1e-5 (mixed);
RDF counts bit-exact; MSD and thermostat draws 1e-12; short trajectories
within the rounding growth of a few tens of steps.
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


def relaxed(n, T=1.0, seed=1, rho=1.2):
    """Oracle-relaxed liquid: (x, y, z, vx, vy, vz, n_a, L)."""
    key = (n, T, seed, rho)
    if key not in _CACHE:
        L = W.box_for(n, rho)
        na = W.n_a_for(n)
        x, y, z = W.lattice_config(n, L, seed, 0.08)
        vx, vy, vz = W.gaussian_velocities(n, math.sqrt(T), seed + 1)
        st = O.State(x, y, z, vx, vy, vz, na, L)
        st.compute_forces()
        O.run(st, 0.001, 150, nb=5, T=T, seed=seed)
        O.run(st, 0.003, 150, nb=10, T=T, seed=seed, step0=150)
        _CACHE[key] = (st.x.copy(), st.y.copy(), st.z.copy(), st.vx.copy(), st.vy.copy(), st.vz.copy(), na, L)
    return _CACHE[key]


def system(configs, precision="fp64", **kw):
    """configs: list of (n, T, seed, rho) relaxed liquids batched in one context."""
    reps, pos, vel = [], [[], [], []], [[], [], []]
    for i, (n, T, seed, rho) in enumerate(configs):
        x, y, z, vx, vy, vz, na, L = relaxed(n, T, seed, rho)
        reps.append((n, na, L, T, 1000 + seed))
        for k, a in enumerate((x, y, z)):
            pos[k].append(a)
        for k, a in enumerate((vx, vy, vz)):
            vel[k].append(a)
    pos = [np.concatenate(p) for p in pos]
    vel = [np.concatenate(v) for v in vel]
    return md.System(reps, precision=precision, positions=pos, velocities=vel, **kw)


def normwise(a, b):
    num = sum(np.sum((a[k] - b[k]) ** 2) for k in range(3))
    den = sum(np.sum(b[k] ** 2) for k in range(3))
    return math.sqrt(num / den)


@pytest.mark.parametrize("n", [500, 2000, 4000])
def test_forces_fp64_match_oracle(n):
    log(f"case forces fp64 n={n}")
    s = system([(n, 1.0, 3, 1.2)], "fp64")
    obs = s.forces(energy=True)
    a = s.numpy()
    x, y, z, _, _, _, na, L = relaxed(n, 1.0, 3)
    fx, fy, fz, pe, w = O.forces(x, y, z, na, L, "brute")
    err = normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz))
    log(f"  normwise {err:.3e}")
    assert err <= 1e-12
    assert obs[0, 0] == pytest.approx(pe, rel=1e-12)
    assert obs[0, 1] == pytest.approx(w, rel=1e-12)
    assert s.status() == 0
    s.close()


@pytest.mark.parametrize("n,skin,cell_div", [(500, 0.2, 1), (500, 0.4, 2), (2000, 0.5, 1), (4000, 0.25, 2),
                                             (1200, 0.0, 1)])
def test_forces_list_parameters(n, skin, cell_div):
    """Pair sets of every list geometry (pruned and unpruned stencils, 1-5
    cells per edge, zero skin) against the O(N^2) oracle."""
    log(f"case list n={n} skin={skin} cell_div={cell_div}")
    for prec, tol in (("fp64", 1e-12), ("mixed_fixed", 1e-5)):
        s = system([(n, 1.0, 25, 1.2)], prec, skin=skin, cell_div=cell_div)
        a = s.numpy()
        x, y, z, _, _, _, na, L = relaxed(n, 1.0, 25)
        fx, fy, fz, _, _ = O.forces(x, y, z, na, L, "brute")
        err = normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz))
        assert err <= tol, (prec, err)
        s.step_nve(100)
        assert s.status() == 0
        s.close()


@pytest.mark.parametrize("prec", ["mixed", "mixed_fixed"])
@pytest.mark.parametrize("n,T", [(2000, 1.0), (4000, 0.5)])
def test_forces_mixed_match_oracle(prec, n, T):
    log(f"case forces {prec} n={n} T={T}")
    s = system([(n, T, 4, 1.2)], prec)
    obs = s.forces(energy=True)
    a = s.numpy()
    x, y, z, _, _, _, na, L = relaxed(n, T, 4)
    fx, fy, fz, pe, w = O.forces(x, y, z, na, L, "cell")
    err = normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz))
    frms = math.sqrt(np.mean(fx ** 2 + fy ** 2 + fz ** 2))
    mx = max(np.max(np.abs(a["ax"] - fx)), np.max(np.abs(a["ay"] - fy)), np.max(np.abs(a["az"] - fz)))
    log(f"  normwise {err:.3e}  max|dF|/Frms {mx / frms:.3e}  PE rel {(obs[0, 0] - pe) / abs(pe):.3e}")
    assert err <= 1e-5
    assert obs[0, 0] == pytest.approx(pe, rel=1e-5)
    assert obs[0, 1] == pytest.approx(w, rel=1e-5)
    assert s.status() == 0
    s.close()


def test_fixed_point_sum_of_forces_is_exactly_zero():
    log("case fixed newton")
    s = system([(4000, 1.0, 5, 1.2), (1500, 0.8, 6, 1.2)], "mixed_fixed")
    a = s.numpy()
    for r in range(2):
        sl = s.replica_slice(r)
        for k in ("ax", "ay", "az"):
            q = np.rint(a[k][sl] * 2.0 ** 26).astype(np.int64)
            assert np.array_equal(q.astype(np.float64) / 2.0 ** 26, a[k][sl])
            assert int(q.sum()) == 0
    s.close()


def test_batched_replicas_match_oracle_per_replica():
    cfgs = [(500, 1.0, 7, 1.2), (3000, 0.6, 8, 1.2), (1200, 1.5, 9, 1.1), (2500, 0.8, 10, 1.3)]
    log("case batched forces", cfgs)
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        s = system(cfgs, prec)
        obs = s.forces(energy=True)
        a = s.numpy()
        for r, (n, T, seed, rho) in enumerate(cfgs):
            x, y, z, _, _, _, na, L = relaxed(n, T, seed, rho)
            fx, fy, fz, pe, w = O.forces(x, y, z, na, L, "brute")
            sl = s.replica_slice(r)
            err = normwise((a["ax"][sl], a["ay"][sl], a["az"][sl]), (fx, fy, fz))
            assert err <= tol, (prec, r, err)
            assert obs[r, 0] == pytest.approx(pe, rel=tol)
        s.close()


def test_nve_fp64_trajectory_matches_oracle():
    n, T = 2000, 1.0
    log("case nve fp64 trajectory")
    s = system([(n, T, 11, 1.2)], "fp64")
    x, y, z, vx, vy, vz, na, L = relaxed(n, T, 11)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    nsteps = 30
    O.run(st, 0.005, nsteps)
    s.step_nve(nsteps)
    a = s.numpy()
    img = s.images()
    ux = a["x"] + img[0] * L
    ox = st.x + st.img[0] * L
    assert np.max(np.abs(ux - ox)) < 1e-9
    assert np.max(np.abs(a["vx"] - st.vx)) < 1e-8
    assert np.array_equal(img, st.img)
    assert s.status() == 0
    s.close()


def test_one_fp64_step_matches_oracle_to_1e13():
    """One velocity-Verlet step (Sec. II.D, in the order of Sec. III.E) in
    FP64 against the oracle's: positions, velocities and the new
    accelerations to 1e-13 relative (normwise; the force sums run in another
    order), image counters equal."""
    n, T = 2000, 1.0
    log("case one fp64 step")
    s = system([(n, T, 12, 1.2)], "fp64")
    x, y, z, vx, vy, vz, na, L = relaxed(n, T, 12)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    O.run(st, 0.005, 1)
    s.step_nve(1)
    a = s.numpy()
    img = s.images()
    assert np.array_equal(img, st.img)

    def rel(keys, ref):
        num = sum(np.sum((a[k] - r) ** 2) for k, r in zip(keys, ref))
        return math.sqrt(num / sum(np.sum(r ** 2) for r in ref))

    ex = rel(("x", "y", "z"), (st.x, st.y, st.z))
    ev = rel(("vx", "vy", "vz"), (st.vx, st.vy, st.vz))
    ea = rel(("ax", "ay", "az"), (st.ax, st.ay, st.az))
    log(f"  positions {ex:.2e}, velocities {ev:.2e}, accelerations {ea:.2e}")
    assert ex <= 1e-13 and ev <= 1e-13 and ea <= 1e-13
    assert s.status() == 0
    s.close()


@pytest.mark.parametrize("n,dr_mode", [(1000, "paper"), (4000, "halfbox200"), (3000, "short"), (6000, "pruned")])
def test_rdf_counts_bit_exact(n, dr_mode):
    """Histogram counts equal the oracle's O(N^2) ones.  "pruned": r_max = 4.0
    in a box of 17.1, where the grid takes cells of half the range (8 per
    edge) and each particle skips the stencil cells beyond r_max."""
    log(f"case rdf n={n} {dr_mode}")
    rho = 1.2
    if dr_mode == "paper":  # N = 1000, L = 9.4, dr = 0.1, n_bins = int(L/2/dr) (Sec. VI.A.1)
        L = 9.4
        rho = n / L ** 3
        dr, nb = 0.1, int(L / 2 / 0.1)
    x, y, z, _, _, _, na, L = relaxed(n, 1.0, 12, rho)
    if dr_mode == "halfbox200":
        dr, nb = (L / 2) / 200, 200
    elif dr_mode == "short":
        dr, nb = 0.02, 150
    elif dr_mode == "pruned":
        dr, nb = 0.1, 40
    s = system([(n, 1.0, 12, rho)], "fp64")
    h = s._host(s.rdf(dr, nb)).astype(np.uint64)[0]
    ref = O.rdf_hist(x, y, z, na, L, dr, nb)
    assert np.array_equal(h, ref), np.argwhere(h != ref)[:5]
    s.close()


def test_msd_matches_oracle():
    n, T = 2000, 1.0
    log("case msd")
    s = system([(n, T, 13, 1.2)], "fp64")
    x, y, z, _, _, _, na, L = relaxed(n, T, 13)
    s.msd_set_origin(2)
    s.step_nve(200)
    got = s.msd(2)[0]
    a = s.numpy()
    img = s.images()
    ref = O.msd(a["x"], a["y"], a["z"], img, na, L, x, y, z)
    assert got == pytest.approx(ref, rel=1e-12)
    assert got[1] > got[0] > 0  # smaller B particles move further
    s.close()


def test_stochastic_bath_draws_match_oracle():
    n, T = 1500, 0.2
    log("case stochastic bath draw")
    s = system([(n, T, 14, 1.2)], "fp64")
    seed = 1000 + 14
    s.step_nvt(10, md.NVT_STOCHASTIC, n_reassign=10)
    a = s.numpy()
    # replica 0, draw tag = step 10, ids = caller index within the replica
    vx, vy, vz = O.mb_velocities(n, T, seed, rep=0, tag=10)
    assert np.max(np.abs(a["vx"] - vx)) < 1e-12
    assert np.max(np.abs(a["vz"] - vz)) < 1e-12
    ke = 0.5 * np.sum(a["vx"] ** 2 + a["vy"] ** 2 + a["vz"] ** 2)
    assert 2 * ke / (3 * n) == pytest.approx(T, rel=1e-13)
    s.close()


def test_nose_hoover_matches_oracle():
    n, T0, T = 1500, 1.0, 0.7
    tau = 0.5
    log("case nose-hoover")
    s = system([(n, T0, 15, 1.2)], "fp64")
    x, y, z, vx, vy, vz, na, L = relaxed(n, T0, 15)
    # the bath temperature is the replica temperature: rebuild with T = 0.7
    s.close()
    s = md.System([(n, na, L, T, 1)], precision="fp64", positions=(x, y, z), velocities=(vx, vy, vz))
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    Q = 3 * n * T * tau ** 2
    e = O.run_nh(st, 0.005, 20, T, Q)
    s.step_nvt(20, md.NVT_NOSE_HOOVER, tau=tau)
    a = s.numpy()
    th = md.md_thermostat_state(s.ctx, 1)[0]
    img = s.images()
    assert np.max(np.abs(a["x"] + img[0] * L - (st.x + st.img[0] * L))) < 1e-9
    assert th[0] == pytest.approx(st.xi, rel=1e-9, abs=1e-12)
    assert th[1] == pytest.approx(st.lns, rel=1e-9, abs=1e-12)
    assert e[-1, 3] == pytest.approx(st.xi)
    s.close()


def _state_equal(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_graph_replay_equals_eager_fixed():
    log("case graph replay")
    cfg = [(3000, 0.8, 16, 1.2)]
    s1 = system(cfg, "mixed_fixed")
    s2 = system(cfg, "mixed_fixed")
    md.md_graph_capture(s2.ctx, 50, 0)
    for _ in range(3):
        s1.step_nve(50)
        md.md_graph_launch(s2.ctx)
        s2.sync()
        assert _state_equal(s1.numpy(), s2.numpy())
    assert s1.status() == 0 and s2.status() == 0
    s1.close()
    s2.close()


def test_graph_replay_stochastic_bath():
    log("case graph stochastic")
    cfg = [(1500, 0.5, 17, 1.2)]
    s1 = system(cfg, "mixed_fixed")
    s2 = system(cfg, "mixed_fixed")
    md.md_graph_capture(s2.ctx, 20, 1, md.NVT_STOCHASTIC, 10)
    for _ in range(2):
        s1.step_nvt(20, md.NVT_STOCHASTIC, 10)
        md.md_graph_launch(s2.ctx)
        s2.sync()
        a, b = s1.numpy(), s2.numpy()
        assert np.max(np.abs(a["vx"] - b["vx"])) < 1e-12
        assert np.max(np.abs(a["x"] - b["x"])) < 1e-12
    s1.close()
    s2.close()


def test_fp64_fused_steps_through_rebuilds_and_redraws():
    """FP64 steps fuse the force with the closing half kick and the next drift,
    except the last step of a call and a step followed by a redraw.  A hot
    liquid (T = 2.0) over 80 steps with a redraw every 9 steps crosses many
    list rebuilds, which reorder the packed positions the fused steps gather,
    and alternates fused and unfused steps; the trajectory follows the
    oracle's stochastic-bath run."""
    n, T, seed = 1500, 2.0, 26
    log("case fp64 fused steps")
    s = system([(n, T, seed, 1.2)], "fp64")
    x, y, z, vx, vy, vz, na, L = relaxed(n, T, seed)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    nsteps, nb = 80, 9
    O.run(st, 0.005, nsteps, nb=nb, T=T, seed=1000 + seed, rep=0)
    r0 = md.md_stats(s.ctx)["rebuilds"]
    s.step_nvt(nsteps, md.NVT_STOCHASTIC, n_reassign=nb)
    assert md.md_stats(s.ctx)["rebuilds"] - r0 >= 3
    a = s.numpy()
    img = s.images()
    assert np.array_equal(img, st.img)
    for k, o in (("x", st.x), ("y", st.y), ("z", st.z)):
        assert np.max(np.abs(a[k] - o)) < 1e-8, k
    for k, o in (("vx", st.vx), ("vy", st.vy), ("vz", st.vz)):
        assert np.max(np.abs(a[k] - o)) < 1e-8, k
    assert s.status() == 0
    s.close()


def test_graph_replay_equals_eager_fp64():
    """Graph replays of fused FP64 steps: each replay packs the positions
    afresh at its first fused step, so replays and eager calls agree bit for
    bit."""
    log("case graph replay fp64")
    cfg = [(2000, 1.5, 27, 1.2)]
    s1 = system(cfg, "fp64")
    s2 = system(cfg, "fp64")
    md.md_graph_capture(s2.ctx, 40, 0)
    for _ in range(3):
        s1.step_nve(40)
        md.md_graph_launch(s2.ctx)
        s2.sync()
        assert _state_equal(s1.numpy(), s2.numpy())
    assert s1.status() == 0 and s2.status() == 0
    s1.close()
    s2.close()


def test_replica_in_batch_equals_alone_fixed():
    log("case batch invariance")
    a_cfg = (2000, 0.9, 18, 1.2)
    batch = [(800, 1.2, 19, 1.2), a_cfg, (3500, 0.6, 20, 1.2)]
    sb = system(batch, "mixed_fixed")
    sa = system([a_cfg], "mixed_fixed")
    sb.step_nve(150)
    sa.step_nve(150)
    ab, aa = sb.numpy(), sa.numpy()
    sl = sb.replica_slice(1)
    for k in aa:
        assert np.array_equal(ab[k][sl], aa[k]), k
    sb.close()
    sa.close()


def test_checkpoint_resume_is_bitwise_fixed():
    log("case checkpoint")
    cfg = [(2500, 0.8, 21, 1.2)]
    s1 = system(cfg, "mixed_fixed")
    s1.step_nve(120)
    ref = s1.numpy()
    s2 = system(cfg, "mixed_fixed")
    s2.step_nve(60)
    blob = md.md_get_state(s2.ctx)
    s3 = system(cfg, "mixed_fixed")
    md.md_set_state(s3.ctx, blob)
    s3.step_nve(60)
    assert _state_equal(ref, s3.numpy())
    for s in (s1, s2, s3):
        s.close()


def test_list_overflow_heals_in_a_graph_replay_by_a_rebuild():
    """Eager calls heal an overflowing list themselves (test_gpu_workspace);
    a graph replay cannot: its steps run on a truncated list and the bit stays
    for md_status.  md_build_cells then grows the list, after which forces
    equal the oracle's again.  (Pairs missing from the truncated lists can
    come too close during the replay; the runaway bit that may then be set
    stays, as every bit but the healed overflow does.)"""
    log("case list overflow in a graph")
    n = 1000
    s = system([(n, 1.0, 22, 1.2)], "fp64", list_capacity=0.05)
    assert s.status() == 0                                  # md_init healed its first build
    rows0 = md.md_stats(s.ctx)["list_rows"]
    # skin 1.0: list radius 3.5 instead of 2.8, about twice the partners, more
    # than the rows the healed skin-0.3 list got (the capacity stays 0.05)
    s.set_list_params(1.0, 1)
    rows1 = md.md_stats(s.ctx)["list_rows"]
    md.md_graph_capture(s.ctx, 20, 0)
    md.md_graph_launch(s.ctx)                               # its first step rebuilds and overflows
    w = s.status()
    log(f"  rows {rows0} -> {rows1}, word 0x{w:x}")
    assert w & md.DEV_LIST_OVERFLOW
    assert w & ~(md.DEV_LIST_OVERFLOW | md.DEV_RUNAWAY) == 0
    s.build_cells()
    assert s.status() == w & md.DEV_RUNAWAY
    assert md.md_stats(s.ctx)["list_rows"] > rows1
    s.forces()
    a = s.numpy()
    fx, fy, fz, _, _ = O.forces(a["x"], a["y"], a["z"], W.n_a_for(n), W.box_for(n, 1.2), "brute")
    assert normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz)) <= 1e-12
    s.close()


def test_rsa_init_and_mb_velocities():
    n = 4000
    log("case rsa init")
    L = W.box_for(n, 1.2)
    s = md.System([(n, W.n_a_for(n), L, 2.0, 77)], precision="fp64", init="rsa", min_dist=0.8)
    a = s.numpy()
    assert O.min_distance(a["x"], a["y"], a["z"], L) >= 0.8 - 1e-12
    assert np.all(a["x"] >= 0) and np.all(a["x"] < L)
    for k in ("vx", "vy", "vz"):
        assert abs(a[k].sum()) < 1e-10
    ke = 0.5 * np.sum(a["vx"] ** 2 + a["vy"] ** 2 + a["vz"] ** 2)
    assert 2 * ke / (3 * n) == pytest.approx(2.0, rel=1e-13)
    # initial forces are those of the positions
    fx, fy, fz, _, _ = O.forces(a["x"], a["y"], a["z"], W.n_a_for(n), L, "cell")
    assert normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz)) < 1e-12
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_fixed"])
def test_nve_energy_drift(prec):
    n, T = 4000, 0.5
    log(f"case drift {prec}")
    s = system([(n, T, 23, 1.2)], prec)
    s.step_nvt(500, md.NVT_STOCHASTIC, 50)
    s.step_nve(200)
    e0 = s.observables()[0, 4]
    es = []
    for _ in range(10):
        s.step_nve(200)
        es.append(s.observables()[0, 4])
    drift = abs(es[-1] - e0) / abs(e0)
    log(f"  E0={e0:.6f} drift over 2000 steps {drift:.2e}")
    assert drift < 1e-4
    assert s.status() == 0
    s.close()


def test_autotune_picks_a_valid_skin():
    log("case autotune")
    s = system([(4000, 0.8, 24, 1.2)], "mixed")
    x0 = s.numpy()["x"].copy()
    res = s.autotune(20)
    assert 0.2 <= res["skin"] <= 0.5 and res["cell_div"] in (1, 2) and res["ms_per_step"] > 0
    s.sync()
    assert np.array_equal(s.numpy()["x"], x0)  # state restored
    s.step_nve(50)
    assert s.status() == 0
    s.close()


def test_set_temperature_redraw_and_nose_hoover_match_oracle():
    """md_set_temperature: the next bath redraw is the oracle's flow chart at
    the new temperature, and a Nose-Hoover run afterwards uses Q = 3 N T tau^2
    at the new T (oracle recurrence, same start)."""
    n, T0, T1 = 1500, 0.2, 0.65
    log("case set temperature")
    s = system([(n, T0, 14, 1.2)], "fp64")
    s.set_temperature(T1)
    s.step_nvt(10, md.NVT_STOCHASTIC, n_reassign=10)
    a = s.numpy()
    vx, vy, vz = O.mb_velocities(n, T1, 1000 + 14, rep=0, tag=10)
    assert np.max(np.abs(a["vx"] - vx)) < 1e-12 and np.max(np.abs(a["vz"] - vz)) < 1e-12
    s.close()
    x, y, z, vx, vy, vz, na, L = relaxed(n, 1.0, 15)
    s = md.System([(n, na, L, 1.0, 1)], precision="fp64", positions=(x, y, z), velocities=(vx, vy, vz))
    s.set_temperature(0.7)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    tau = 0.5
    O.run_nh(st, 0.005, 20, 0.7, 3 * n * 0.7 * tau ** 2)
    s.step_nvt(20, md.NVT_NOSE_HOOVER, tau=tau)
    th = md.md_thermostat_state(s.ctx, 1)[0]
    assert th[0] == pytest.approx(st.xi, rel=1e-9, abs=1e-12)
    assert th[1] == pytest.approx(st.lns, rel=1e-9, abs=1e-12)
    with pytest.raises(md.KamdError):
        s.set_temperature(-1.0)
    s.close()


def test_scale_velocities_per_replica():
    log("case scale velocities")
    s = system([(800, 1.0, 21, 1.2), (1200, 0.6, 22, 1.2)], "fp64")
    a0 = s.numpy()
    o0 = s.observables()
    f = np.array([1.25, 0.5])
    s.scale_velocities(f)
    a1 = s.numpy()
    o1 = s.observables()
    for i in range(2):
        sl = s.replica_slice(i)
        for k in ("vx", "vy", "vz"):
            assert np.array_equal(a1[k][sl], a0[k][sl] * f[i])
        for k in ("x", "ax"):
            assert np.array_equal(a1[k][sl], a0[k][sl])
    assert np.allclose(o1[:, 0], o0[:, 0] * f ** 2, rtol=1e-13)
    assert np.array_equal(o1[:, 1], o0[:, 1])
    s.close()


def test_temperature_ladder_end_to_end():
    """Four independent ladders (replicas) through T = 2.0 and 1.0 with energy
    rescaling: the MSD grows,
    D decreases with T, and B particles diffuse faster than A (Sec. V)."""
    from paper_2001_07089_amd import ladder
    log("case temperature ladder")
    s = system([(1000, 2.0, 31 + r, 1.2) for r in range(4)], "mixed_fixed")
    stages = [ladder.Stage(2.0, 400, 3000), ladder.Stage(1.0, 400, 3000)]
    res = ladder.run_ladder(s, stages, 0.005, rescale_energy=True)
    for r in res:
        assert np.all(np.diff(r.msd[:, :, 0], axis=0)[-10:] > 0)
        assert np.all(r.diffusion > 0)
    d2, d1 = res[0].diffusion.mean(axis=0), res[1].diffusion.mean(axis=0)
    log(f"  D(2.0) = {d2}, D(1.0) = {d1}")
    assert d2[0] > d1[0] and d2[1] > d1[1]
    assert d1[1] > d1[0]
    assert s.status() == 0
    s.close()


def test_van_hove_self_matches_oracle_bit_exact():
    """Self van Hove histogram against an MSD origin, two replicas, FP64:
    counts equal the oracle's for every bin."""
    log("case van hove")
    cfgs = [(1200, 1.0, 41, 1.2), (800, 0.8, 42, 1.2)]
    s = system(cfgs, "fp64")
    a0 = s.numpy(("x", "y", "z"))
    img0 = s.images()
    s.msd_set_origin(2)
    s.step_nve(60)
    a = s.numpy(("x", "y", "z"))
    img = s.images()
    dr, nb = 0.01, 400
    h = s._host(s.van_hove(2, dr, nb)).astype(np.uint64)
    for i, (n, T, seed, rho) in enumerate(cfgs):
        sl = s.replica_slice(i)
        L = W.box_for(n, rho)
        na = W.n_a_for(n)
        u0 = O.unwrapped(a0["x"][sl], a0["y"][sl], a0["z"][sl], img0[:, sl], L)
        ref = O.van_hove_self(a["x"][sl], a["y"][sl], a["z"][sl], np.ascontiguousarray(img[:, sl]), na, L,
                              *u0, dr, nb)
        assert np.array_equal(h[i], ref), i
        assert int(h[i][0].sum()) == na and int(h[i][1].sum()) == n - na
    with pytest.raises(md.KamdError):
        s.van_hove(2, dr, 5000)
    s.close()


def test_quench_aging_two_time_msd():
    """Instant quench T = 2.0 -> 0.3: younger systems move more over the same
    lag (two-time MSD, Eq. (msdtw)); the van Hove histograms at each point
    hold every particle."""
    from paper_2001_07089_amd import aging
    log("case quench aging")
    s = system([(1000, 2.0, 51 + r, 1.2) for r in range(4)], "mixed_fixed")
    out = aging.quench(s, 0.3, 1000, t_w=(0, 10, 100, 500), van_hove=(0.02, 1024))
    def at(tw, lag):
        k = int(np.searchsorted(out[tw].lags, lag))
        assert out[tw].lags[k] == lag
        return out[tw].msd[k].mean(axis=0)
    common = np.intersect1d(out[0].lags, out[500].lags)  # the two schedules differ (n_MD differs)
    lag = int(common[np.argmin(np.abs(common - 100))])
    m0, m500 = at(0, lag), at(500, lag)
    log(f"  msd(t_w=0, lag {lag}) = {m0}, msd(t_w=500) = {m500}")
    assert m0[0] > m500[0] and m0[1] > m500[1]
    vh = out[10].van_hove
    assert vh.shape[1:] == (4, 2, 1024)
    assert np.all(vh[:, :, 0, :].sum(axis=-1) == W.n_a_for(1000))
    assert s.status() == 0
    s.close()


_PLANAR = {}


def planar_relaxed(n=1000, T=0.4, seed=3):
    """Oracle-relaxed planar 65:35 liquid at N/L^2 = 1.204 (z = vz = 0)."""
    key = (n, T, seed)
    if key not in _PLANAR:
        wl = W.ka_planar(n, T)
        r = wl.replicas[0]
        x, y, z = W.planar_lattice_config(n, r.box, seed)
        vx, vy, vz = O.mb_velocities(n, T, seed, dim=2)
        st = O.State(x, y, z, vx, vy, vz, r.n_a, r.box)
        st.compute_forces()
        O.run(st, 0.00025, 300, nb=5, T=T, seed=seed, dim=2)
        O.run(st, 0.002, 1500, nb=10, T=T, seed=seed, dim=2, step0=300)
        _PLANAR[key] = (st.x.copy(), st.y.copy(), st.z.copy(), st.vx.copy(), st.vy.copy(), st.vz.copy(),
                        r.n_a, r.box)
    return _PLANAR[key]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed_fixed", 1e-5)])
def test_planar_forces_match_oracle(prec, tol):
    n = 1000
    x, y, z, vx, vy, vz, na, L = planar_relaxed(n)
    log(f"case planar forces {prec}")
    s = md.System([(n, na, L, 0.4, 5)], precision=prec, positions=(x, y, z), velocities=(vx, vy, vz), dim=2)
    a = s.numpy(("ax", "ay", "az"))
    fx, fy, fz, pe, _ = O.forces(x, y, z, na, L, "brute")
    assert np.all(a["az"] == 0.0) and np.all(fz == 0.0)
    assert normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz)) <= tol
    assert s.forces(energy=True)[0, 0] == pytest.approx(pe, rel=max(tol, 1e-12))
    s.close()


def test_planar_bath_nve_and_nose_hoover_match_oracle():
    """Planar system: the bath redraw is the oracle's planar flow chart
    (vz = 0, sum v^2 = 2 N T), NVE steps follow the oracle's trajectory and
    stay in the plane, Nose-Hoover uses X = 2N."""
    n, T = 1000, 0.4
    x, y, z, vx, vy, vz, na, L = planar_relaxed(n, T)
    log("case planar dynamics")
    s = md.System([(n, na, L, T, 77)], precision="fp64", positions=(x, y, z), velocities=(vx, vy, vz), dim=2)
    s.step_nvt(10, md.NVT_STOCHASTIC, n_reassign=10)
    a = s.numpy()
    rx, ry, rz = O.mb_velocities(n, T, 77, rep=0, tag=10, dim=2)
    assert np.all(a["vz"] == 0.0) and np.all(a["z"] == 0.0)
    assert np.max(np.abs(a["vx"] - rx)) < 1e-12 and np.max(np.abs(a["vy"] - ry)) < 1e-12
    assert s.observables()[0, 3] == pytest.approx(T, rel=1e-12)  # T = 2 KE / (2 N)
    s.close()
    s = md.System([(n, na, L, T, 77)], precision="fp64", positions=(x, y, z), velocities=(vx, vy, vz), dim=2,
                  dt=0.002)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    O.run(st, 0.002, 40)
    s.step_nve(40)
    a = s.numpy()
    img = s.images()
    assert np.all(a["z"] == 0.0) and np.all(img[2] == 0)
    assert np.max(np.abs(a["x"] + img[0] * L - (st.x + st.img[0] * L))) < 1e-9
    assert np.max(np.abs(a["vy"] - st.vy)) < 1e-9
    s.close()
    s = md.System([(n, na, L, T, 77)], precision="fp64", positions=(x, y, z), velocities=(vx, vy, vz), dim=2,
                  dt=0.002)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    tau = 0.3
    O.run_nh(st, 0.002, 20, 0.3, 2 * n * 0.3 * tau ** 2, dim=2)
    s.set_temperature(0.3)
    s.step_nvt(20, md.NVT_NOSE_HOOVER, tau=tau)
    th = md.md_thermostat_state(s.ctx, 1)[0]
    assert th[0] == pytest.approx(st.xi, rel=1e-9, abs=1e-12)
    s.close()


def test_planar_rsa_init_and_rdf():
    wl = W.ka_planar()
    r = wl.replicas[0]
    log("case planar rsa + rdf")
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="mixed", init="rsa", dim=2)
    a = s.numpy()
    assert np.all(a["z"] == 0.0) and np.all(a["vz"] == 0.0)
    assert O.min_distance(a["x"], a["y"], a["z"], r.box) >= 0.8 - 1e-12
    assert s.observables()[0, 3] == pytest.approx(r.temperature, rel=1e-12)
    dr = 0.05
    nb = int(r.box / 2 / dr)
    h = s._host(s.rdf(dr, nb)).astype(np.uint64)[0]
    assert np.array_equal(h, O.rdf_hist(a["x"], a["y"], a["z"], r.n_a, r.box, dr, nb))
    s.step_nve(200)
    assert s.status() == 0 and np.all(s.numpy(("z",))["z"] == 0.0)
    s.close()


# ------------------------------------------ LAMMPS conventions (Sec. IV.B, VI.A.3)

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed_fixed", 1e-5)])
def test_unshifted_energy_matches_oracle_and_forces_are_unchanged(prec, tol):
    """pe_unshifted: the potential energy of LAMMPS lj/cut (no V_ab(r_c)
    term) against the oracle's brute-force sum; the forces are bit for bit
    those of the shifted configuration."""
    n = 2000
    log(f"case unshifted energy {prec}")
    x, y, z, _, _, _, na, L = relaxed(n, 1.0, 3)
    shifted = system([(n, 1.0, 3, 1.2)], prec)
    cut = system([(n, 1.0, 3, 1.2)], prec, pe_unshifted=True)
    o_s = shifted.forces(energy=True)
    o_c = cut.forces(energy=True)
    a_s = shifted.numpy(("ax", "ay", "az"))
    a_c = cut.numpy(("ax", "ay", "az"))
    for k in ("ax", "ay", "az"):
        assert np.array_equal(a_s[k], a_c[k])
    assert o_c[0, 0] == pytest.approx(O.pe_lj_cut(x, y, z, na, L), rel=max(tol, 1e-12))
    assert o_c[0, 1] == o_s[0, 1]  # virial unchanged
    ob_s, ob_c = shifted.observables()[0], cut.observables()[0]
    assert ob_c[4] - ob_s[4] == pytest.approx(o_c[0, 0] - o_s[0, 0], rel=1e-12)  # E_tot moves with PE
    shifted.close()
    cut.close()


def test_lammps_rdf_table_from_device_counts():
    """compute rdf 25 bins to the force cutoff 2.5: the device counts equal the
    oracle's, and the table (g, coordination numbers) equals the oracle's."""
    from paper_2001_07089_amd import analysis
    n = 3000
    log("case lammps rdf")
    x, y, z, _, _, _, na, L = relaxed(n, 1.0, 4)
    s = system([(n, 1.0, 4, 1.2)], "fp64")
    rcut, nbins = 2.5, 25
    h = s._host(s.rdf(rcut / nbins, nbins)).astype(np.uint64)[0]
    ref = O.rdf_hist(x, y, z, na, L, rcut / nbins, nbins)
    assert np.array_equal(h, ref)
    t = analysis.lammps_rdf(h, n, na, L, rcut)
    assert np.allclose(t, O.lammps_rdf_table(ref, n, na, L, rcut, nbins), rtol=1e-13, atol=0.0)
    # partners within 2.5: about rho_J * 4 pi 2.5^3 / 3, i.e. ~63 A and ~16 B around an A
    assert 50.0 < t[-1, 3] < 75.0 and 10.0 < t[-1, 7] < 22.0
    s.close()


def test_lammps_data_file_round_trip_through_the_device():
    """A replica written as a LAMMPS data file and read back starts a new
    context whose forces and state equal the original bit for bit."""
    import io
    from paper_2001_07089_amd import lammps_io as LIO
    n = 1500
    log("case lammps data round trip")
    s = system([(n, 0.8, 6, 1.2)], "mixed_fixed")
    s.step_nve(37)
    arr = LIO.replica_arrays(s, 0)
    buf = io.StringIO()
    LIO.write_data(buf, arr["x"], arr["y"], arr["z"], arr["n_a"], arr["L"], arr["vx"], arr["vy"], arr["vz"],
                   img=arr["img"])
    got = LIO.read_data(io.StringIO(buf.getvalue()))
    s2 = md.System([(got["n"], got["n_a"], got["L"], 0.8, 1006)], precision="mixed_fixed",
                   positions=(got["x"], got["y"], got["z"]), velocities=(got["vx"], got["vy"], got["vz"]))
    s.forces()
    s2.forces()
    a, b = s.numpy(), s2.numpy()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    s.close()
    s2.close()


def test_list_statistics_count_16bit_entries():
    """A 2000-particle box has fewer than 2^16 slots per type segment, so the
    own-type part of every list is stored in 16 bits and the other part in
    32: about 0.8 * 2 + 0.2 * 4 bytes per partner for A particles and
    0.2 * 2 + 0.8 * 4 for B, 2.6 on average."""
    log("case list statistics")
    s = system([(2000, 1.0, 3, 1.2)], "mixed_fixed")
    md.md_set_force_kernel(s.ctx, 0)          # slot-index entries
    s.forces()
    st = md.md_stats(s.ctx)
    ratio = st["mean_list_bytes"] / st["mean_list_len"]
    log(f"  bytes per partner {ratio:.3f}")
    assert 2.3 < ratio < 3.0
    assert st["max_list_len"] <= st["list_rows"]
    # every lane walks its partners, its own slot and the padding up to the
    # wavefront's longest part
    assert st["mean_list_len"] + 1 <= st["mean_walked"] <= 2 * st["list_rows"]
    assert st["windows"] == 0 and st["staged_fraction"] == 0
    # window entries are 16-bit offsets: 2 bytes per partner in a part whose
    # window fits, so staging can only lower the bytes per partner
    md.md_set_force_kernel(s.ctx, 1)
    s.forces()
    st = md.md_stats(s.ctx)
    log(f"  staged fraction {st['staged_fraction']:.3f}")
    assert st["windows"] == 1 and 0.0 < st["staged_fraction"] <= 1.0
    r1 = st["mean_list_bytes"] / st["mean_list_len"]
    assert 2.0 <= r1 <= ratio + 1e-9
    if st["staged_fraction"] == 1.0:
        assert r1 == pytest.approx(2.0)
    s.close()


@pytest.mark.parametrize("n,rho", [(4000, 1.2), (3020, 1.2), (3000, 0.02), (3000, 2.5e-4)])
def test_list_holds_every_pair_within_the_list_radius(n, rho):
    """Every ordered pair closer than its list radius r_c,ab + skin (Sec. III.C)
    is in the Verlet list, and few others are.  The boxes of 14.9, 13.6 and
    53.1 use the list builder's candidate test on coordinates cut to 16 bits;
    the box of 228.9 uses the full 32-bit test.  The box of 13.6 has 4 cells
    per edge at skin 0.3 and 5 at the skin it builds with (0.22, reported as
    skin_min); the box of 53.1 trims its skin to 0.296 (18 -> 19 cells).
    Exact pair counts: the oracle's O(N^2) distance histogram, one per pair
    type, with 100 bins up to that type's list radius."""
    skin = 0.3
    L = W.box_for(n, rho)
    na = W.n_a_for(n)
    log(f"case list superset n={n} rho={rho} L={L:.1f}")
    s = md.System([(n, na, L, 1.0, 41)], precision="mixed_fixed", init="rsa", min_dist=0.8, skin=skin)
    s.forces()
    assert s.status() == 0
    a = s.numpy(("x", "y", "z"))
    st = md.md_stats(s.ctx)
    s.close()
    used = st["skin_min"]
    assert 2 * skin / 3 <= used <= skin
    if n == 3020:
        assert 0.2 <= used < 0.25
    # hist rows AA, AB, BB: same-type pairs counted twice, AB pairs once
    exact = 0
    for p, mult in ((0, 1), (1, 2), (2, 1)):
        rl = O.KA_RC_FACTOR * O.KA_SIGMA[p] + used
        h = O.rdf_hist(a["x"], a["y"], a["z"], na, L, rl / 100, 100).astype(np.int64)
        exact += mult * int(h[p].sum())
    listed = int(round(st["mean_list_len"] * n))
    log(f"  skin {used:.4f}, exact {exact} listed {listed}")
    assert exact <= listed <= exact * 1.004 + 8
