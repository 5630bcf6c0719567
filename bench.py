"""Throughput benchmark of the Kob-Andersen MD hot path on one MI355X.

Default workload: N = 1,048,576 Kob-Andersen particles (80:20) at density
1.2 and T = 0.45, dt = 0.005, mixed precision with 64-bit fixed-point force
accumulation.  Set-up (not timed): simple-cubic lattice with B/A swaps,
Maxwell-Boltzmann velocities, stochastic-bath equilibration, neighbour-list
autotuning, warm-up steps.  Timed: K velocity-Verlet NVE steps replayed from a
captured HIP graph (forces, integration and every neighbour-list rebuild
included).  One JSON line on stdout.

Also measured (reported in extra keys): the plain FP64 GPU path on the same
workload, the energy drift of the timed window, the force kernel's mean
duration from HIP events (roofline) and the FP64 CPU oracle on a bounded
sample (cpu_baseline).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 19          # FP32 FLOPs per in-cutoff pair force (FMA = 2)
# FP32 vector peak without packed-FP32 instructions (the library is compiled
# without them): 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz.  The published 157.3
# TFLOP/s counts packed FP32 (two FMAs per lane per cycle).
FP32_VECTOR_PEAK = 78.6     # TFLOP/s
FP32_VECTOR_PEAK_PACKED = 157.3
HBM_PEAK = 8000.0           # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kernel_hbm_traffic.md")
TRAFFIC_SOURCES = ("paper_2001_07089_amd/csrc/kernels_force.hip", "paper_2001_07089_amd/csrc/common_dev.hpp",
                   "paper_2001_07089_amd/csrc/kamd_internal.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    p.add_argument("--precision", default="mixed_fixed", choices=["fp64", "mixed", "mixed_fixed"])
    p.add_argument("--equil", type=int, default=6000, help="stochastic-bath steps before timing")
    p.add_argument("--no-autotune", action="store_true")
    p.add_argument("--skin", type=float, default=None, help="fixed list skin (skips the autotuner)")
    p.add_argument("--cell-div", type=int, default=1, help="cell division with --skin")
    p.add_argument("--no-analysis", action="store_true", help="skip the RDF / MSD timings")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison run")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--profile-steps", type=int, default=200)
    p.add_argument("--no-batch", action="store_true", help="skip the batched-replica leg")
    p.add_argument("--batch-steps", type=int, default=1000)
    p.add_argument("--planar", action="store_true",
                   help="also run the planar KA variant (65:35, N/L^2 = 1.204) at N = 2^20, T = 0.4")
    p.add_argument("--ladder", action="store_true",
                   help="also run a temperature ladder: 64 independent N=1000 ladders through T = 3.0 ... 0.5")
    p.add_argument("--batch-large", action="store_true",
                   help="also run the 64-replica batch (N 50k-500k each, ~17.6M particles) with admission, "
                        "RDF and MSD sampling")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB (5 times) and exit: the reference "
                        "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def make_system(wl, precision, md):
    rep = wl.replicas[0]
    init = "rsa" if rep.n <= 300000 else "lattice"
    return md.System([(rep.n, rep.n_a, rep.box, rep.temperature, rep.seed)], precision=precision,
                     dt=wl.dt, skin=0.3, init=init, auto_sync=False), init


def equilibrate(s, md, nsteps):
    if nsteps <= 0:
        return
    # melt/thermalise with frequent redraws first, then the paper's ~50-step bath
    s.step_nvt(min(500, nsteps), md.NVT_STOCHASTIC, n_reassign=10)
    if nsteps > 500:
        s.step_nvt(nsteps - 500, md.NVT_STOCHASTIC, n_reassign=50)
    w = s.status()
    if w:
        raise RuntimeError(f"device error word 0x{w:x} during equilibration")


def timed_graph(s, md, torch, steps):
    md.md_graph_capture(s.ctx, steps, 0)
    md.md_graph_launch(s.ctx)  # warm replay (also checks the graph)
    s.stream.synchronize()
    e0 = s.observables()[0, 4]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    md.md_graph_launch(s.ctx)
    s.stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e1 = s.observables()[0, 4]
    return t1 - t0, e0, e1


# Bytes per particle that the force launch must move besides its list: for
# the fused mixed-precision step (forces, closing half kick, next drift) it
# reads x,y,z,vx,vy,vz (48), the image counters (12), the u32 mirror (16) and
# the mirror at the last list build (16), and writes x..vz (48), the image
# counters (12) and the next mirror (16); the FP64 force-only kernel reads
# x,y,z (24) and writes ax,ay,az (24).  The list adds its stored size: a
# 4-byte index per entry, or a 2-byte offset where the part of the list is
# stored in 16 bits (md_stats mean_list_bytes, without wavefront padding).
STATE_BYTES = {"mixed": 168, "mixed_fixed": 168, "fp64": 48}


def algorithmic_bytes(mean_list_bytes, n, precision):
    return n * (mean_list_bytes + STATE_BYTES[precision])


def kernel_name(precision):
    return {"fp64": "k_force_fp64<false>", "mixed": "k_force_mixed<false,false,true>",
            "mixed_fixed": "k_force_mixed<true,false,true>"}[precision]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(skin, cell_div, precision, n):
    """HBM bytes per launch of the force kernel from the committed counter
    summary, when it was taken on the current kernel source at the same list
    parameters, precision and size; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    try:
        ok = (kv["source_digest"] == source_digest() and abs(float(kv["skin"]) - skin) < 1e-9
              and int(kv["cell_div"]) == cell_div and kv["precision"] == precision and int(kv["n_atoms"]) == n)
        return float(kv["hbm_bytes_per_launch"]) if ok else None
    except (KeyError, ValueError):
        return None


def time_analysis(s, md, rep):
    """On-device RDF (r_max 5.0, 200 bins) and MSD (one origin, one measurement)
    of the large system, each timed on its own (wall clock around a synced call)."""
    import torch
    dr = 5.0 / 200
    s.rdf(dr, 200)  # warm (allocates the histogram grid)
    s.stream.synchronize()
    t0 = time.perf_counter()
    h = s.rdf(dr, 200)
    s.stream.synchronize()
    t_rdf = time.perf_counter() - t0
    counts = s._host(h).astype(np.int64)[0].sum(axis=1)
    # the LAMMPS compute rdf layout: 25 bins to the force cutoff 2.5, with
    # coordination numbers (host normalisation of the device counts)
    from paper_2001_07089_amd import analysis
    s.rdf(2.5 / 25, 25)
    s.stream.synchronize()
    t0 = time.perf_counter()
    h25 = s.rdf(2.5 / 25, 25)
    table = analysis.lammps_rdf(s._host(h25)[0], rep.n, rep.n_a, rep.box, 2.5)
    t_lmp = time.perf_counter() - t0
    s.msd_set_origin(1)
    s.step_nve(100)
    s.stream.synchronize()
    t0 = time.perf_counter()
    m = s.msd(1)
    t_msd = time.perf_counter() - t0
    torch.cuda.synchronize()
    return {"rdf_ms": t_rdf * 1e3, "rdf_r_max": 5.0, "rdf_bins": 200,
            "rdf_pair_counts_AA_AB_BB": [int(c) for c in counts],
            "lammps_rdf_ms": t_lmp * 1e3, "lammps_rdf_coordination_at_2.5_AA_BB_AB":
                [float(table[-1, 3]), float(table[-1, 5]), float(table[-1, 7])],
            "msd_ms": t_msd * 1e3, "msd_after_100_steps_A_B": [float(m[0, 0]), float(m[0, 1])]}


def cpu_baseline(wl, seconds):
    import oracle as O
    from paper_2001_07089_amd import workload as W
    rep = wl.replicas[0]
    x, y, z = W.lattice_config(rep.n, rep.box, rep.seed, 0.1)
    vx, vy, vz = W.gaussian_velocities(rep.n, math.sqrt(rep.temperature), rep.seed + 1)
    st = O.State(x, y, z, vx, vy, vz, rep.n_a, rep.box)
    t0 = time.perf_counter()
    st.compute_forces("cell")
    tf = time.perf_counter() - t0
    nsteps = max(1, min(200, int(seconds / max(tf, 1e-6))))
    t0 = time.perf_counter()
    O.run(st, wl.dt, nsteps, method="cell")
    el = time.perf_counter() - t0
    return {"value": rep.n * nsteps / el, "unit": "atom-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{nsteps} velocity-Verlet NVE steps of the same N={rep.n} system "
                      f"(cell-list oracle, FP64, OpenMP), {el:.1f} s"}


def batched(md, torch, W, steps):
    """256 replicas, N uniform on [250, 8000], T on [0.45, 2.0], mixed precision:
    one launch per kernel per step over all replicas, HIP-graph replay."""
    wl = W.ka_batch_small()
    reps = [(r.n, r.n_a, r.box, r.temperature, r.seed) for r in wl.replicas]
    t0 = time.perf_counter()
    s = md.System(reps, precision="mixed", dt=wl.dt, skin=0.3, init="rsa", auto_sync=False)
    log(f"batch init (rsa, {len(reps)} replicas, {wl.n_total} particles) {time.perf_counter() - t0:.1f} s")
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(1500, md.NVT_STOCHASTIC, n_reassign=50)
    tune = s.autotune(60)
    s.step_nve(200)
    s.stream.synchronize()
    md.md_graph_capture(s.ctx, steps, 0)
    md.md_graph_launch(s.ctx)
    s.stream.synchronize()
    obs0 = s.observables()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    md.md_graph_launch(s.ctx)
    s.stream.synchronize()
    el = time.perf_counter() - t1
    obs1 = s.observables()
    w = s.status()
    drift = np.abs(obs1[:, 4] - obs0[:, 4]) / np.abs(obs0[:, 4]) * (1e4 / steps)
    out = {"workload": wl.name, "n_replicas": len(reps), "n_atoms": wl.n_total, "precision": "mixed",
           "steps": steps, "value": wl.n_total * steps / el, "unit": "atom-steps/s",
           "ms_per_step": el * 1e3 / steps, "max_drift_per_1e4": float(drift.max()),
           "median_drift_per_1e4": float(np.median(drift)), "autotune": tune, "device_error_word": w}
    s.close()
    return out


def batched_large(md, torch, W):
    """64 replicas, N uniform on [5e4, 5e5], density in {1.1, 1.2, 1.3}, T on
    [0.45, 1.0], MIXED: admission against the free device memory, lattice
    start, 1000 stochastic-bath steps, then 1000 NVE steps replayed from a
    graph in four blocks of 250 with an RDF sample (r_max 5.0, 200 bins) and
    an MSD origin at the start of each block.  The NVE steps are timed; the
    RDF and MSD calls are timed on their own."""
    wl = W.ka_batch_large()
    reps_all = md.make_replicas([(r.n, r.n_a, r.box, r.temperature, r.seed) for r in wl.replicas])
    cfg = md.make_config("mixed", wl.dt, 0.3, md.INIT_LATTICE)
    free, _ = torch.cuda.mem_get_info()
    adm, cnt = md.md_admit(cfg, reps_all, int(free * 0.8))
    chosen = [r for r, a in zip(wl.replicas, adm) if a]
    reps = [(r.n, r.n_a, r.box, r.temperature, r.seed) for r in chosen]
    n_tot = sum(r.n for r in chosen)
    t0 = time.perf_counter()
    s = md.System(reps, precision="mixed", dt=wl.dt, skin=0.3, init="lattice", auto_sync=False)
    log(f"batch-large init ({cnt} of {len(wl.replicas)} replicas admitted, {n_tot} particles) "
        f"{time.perf_counter() - t0:.1f} s")
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=50)
    dr = 5.0 / 200
    s.rdf(dr, 200)  # allocates the histogram grid (a reallocation would drop a captured graph)
    s.stream.synchronize()
    md.md_graph_capture(s.ctx, 250, 0)
    obs0 = s.observables()
    t_nve = t_rdf = t_msd = 0.0
    for blk in range(4):
        t1 = time.perf_counter()
        s.msd_set_origin(blk)
        s.rdf(dr, 200)
        s.stream.synchronize()
        t_rdf += time.perf_counter() - t1
        t1 = time.perf_counter()
        md.md_graph_launch(s.ctx)
        s.stream.synchronize()
        t_nve += time.perf_counter() - t1
    t1 = time.perf_counter()
    msd = [s.msd(k) for k in range(4)]
    t_msd = time.perf_counter() - t1
    obs1 = s.observables()
    drift = np.abs(obs1[:, 4] - obs0[:, 4]) / np.abs(obs0[:, 4]) * (1e4 / 1000)
    out = {"workload": wl.name, "n_replicas_admitted": cnt, "n_replicas": len(wl.replicas), "n_atoms": n_tot,
           "precision": "mixed", "nve_steps": 1000, "value": n_tot * 1000 / t_nve, "unit": "atom-steps/s",
           "ms_per_step": t_nve * 1e3 / 1000, "rdf_ms_per_sample": t_rdf * 1e3 / 4,
           "msd_ms_per_measurement": t_msd * 1e3 / 4, "max_drift_per_1e4": float(drift.max()),
           "median_drift_per_1e4": float(np.median(drift)),
           "msd_A_after_1000_steps_median": float(np.median(msd[0][:, 0])), "device_error_word": s.status()}
    s.close()
    return out


def planar_leg(md, torch, W, steps=1000):
    """The planar KA variant of the appendix exercise at N = 2^20: square
    lattice start, 12,000 bath steps at T = 0.4 with a redraw every 10 steps
    (the strained lattice keeps releasing heat for many thousand steps; a
    shorter or weaker bath leaves a relaxing system whose NVE energy drifts in
    FP64 as much as here), then graph-replayed NVE steps timed."""
    wl = W.ka_planar(1 << 20, 0.4)
    r = wl.replicas[0]
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="mixed_fixed", dt=wl.dt, skin=0.3,
                  init="lattice", auto_sync=False, dim=2)
    s.step_nvt(12000, md.NVT_STOCHASTIC, n_reassign=10)
    tune = s.autotune(100)
    s.step_nve(200)
    el, e0, e1 = timed_graph(s, md, torch, steps)
    out = {"workload": wl.name, "n_atoms": r.n, "box": r.box, "value": r.n * steps / el, "unit": "atom-steps/s",
           "ms_per_step": el * 1e3 / steps, "drift_per_1e4": abs(e1 - e0) / abs(e0) * (1e4 / steps),
           "bath_steps": 12000, "T_after": float(s.observables()[0, 3]),
           "autotune": tune, "device_error_word": s.status()}
    s.close()
    return out


def ladder_leg(md, W):
    """64 independent ladders (replicas) of the paper's N = 1000, L = 9.41
    system through T = 3.0, 2.0, 1.0, 0.8, 0.6, 0.55, 0.5: stochastic bath,
    energy rescale, NVE equilibration, NVE production with log-spaced MSD and
    a fit of D_A, D_B (mean over ladders).  Whole-sequence throughput."""
    from paper_2001_07089_amd import ladder
    wl = W.ka_small()
    r0 = wl.replicas[0]
    reps = [(r0.n, r0.n_a, r0.box, 3.0, r0.seed + 17 * k) for k in range(64)]
    s = md.System(reps, precision="mixed_fixed", dt=wl.dt, skin=0.3, init="rsa", auto_sync=False)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    stages = [ladder.Stage(T, 2000, 10000) for T in (3.0, 2.0, 1.0, 0.8, 0.6, 0.55, 0.5)]
    t0 = time.perf_counter()
    res = ladder.run_ladder(s, stages, wl.dt, rescale_energy=True)
    el = time.perf_counter() - t0
    steps = sum(2 * st.n_equil + st.n_prod for st in stages)
    n_tot = 64 * r0.n
    out = {"ladders": 64, "n_per_ladder": r0.n, "steps": steps, "value": n_tot * steps / el, "unit": "atom-steps/s",
           "seconds": el, "D_A_B_by_T": {f"{r.temperature}": [float(x) for x in r.diffusion.mean(axis=0)]
                                          for r in res},
           "device_error_word": s.status()}
    s.close()
    return out


def calibrate_copy(torch, mib):
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {mib} MiB x 5")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path (asked for {a.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2001_07089_amd import md
    from paper_2001_07089_amd import workload as W

    if a.calibrate_copy:
        calibrate_copy(torch, a.calibrate_copy)
        return

    wl = {"small": W.ka_small, "medium": W.ka_medium, "large": W.ka_large}[a.workload]()
    rep = wl.replicas[0]
    n = rep.n
    log(f"workload {wl.name}: N={n} L={rep.box:.6f} T={rep.temperature} precision={a.precision}")

    t0 = time.perf_counter()
    s, init = make_system(wl, a.precision, md)
    log(f"init ({init}) {time.perf_counter() - t0:.1f} s")
    # melt the start, tune the list on the liquid, then equilibrate at the
    # tuned list parameters (so nearly every force launch of the run, and of
    # a kernel trace of it, uses them)
    first = min(1000, a.equil)
    equilibrate(s, md, first)
    tune = None
    if a.skin is not None:
        s.set_list_params(a.skin, a.cell_div)
        log(f"list parameters fixed: skin {a.skin}, cell_div {a.cell_div}")
    elif not a.no_autotune:
        tune = s.autotune(100)
        log(f"autotune: {tune}")
    if a.equil > first:
        s.step_nvt(a.equil - first, md.NVT_STOCHASTIC, n_reassign=50)
    log(f"equilibrated {a.equil} steps, {time.perf_counter() - t0:.1f} s")
    s.step_nve(a.warmup)
    s.stream.synchronize()
    el, e0, e1 = timed_graph(s, md, torch, a.steps)
    value = n * a.steps / el
    drift = abs(e1 - e0) / abs(e0) * (1e4 / a.steps)
    log(f"timed {a.steps} steps: {el * 1e3:.1f} ms -> {value:.4e} atom-steps/s, "
        f"E/N {e0 / n:.6f} -> {e1 / n:.6f}, drift per 1e4 steps {drift:.2e}")
    prof = md.md_profile(s.ctx, a.profile_steps)
    st = md.md_stats(s.ctx)
    w = s.status()
    log(f"profile: {prof}")
    log(f"stats: {st}  err=0x{w:x}")
    skin = st["skin"]
    pairs = prof["pairs"]
    flops = pairs * FLOP_PER_PAIR
    achieved = flops / (prof["force_ms"] * 1e-3) / 1e12
    candidates = st["mean_list_len"] * n
    traffic = stored_traffic(skin, int(st["cell_div"]), a.precision, n)
    alg = algorithmic_bytes(st["mean_list_bytes"], n, a.precision)
    gbs = alg / (prof["force_ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": gbs / HBM_PEAK,
            "traffic": traffic, "kernel": kernel_name(a.precision), "kernel_ms": prof["force_ms"],
            "algorithmic_bytes_per_launch": alg,
            "traffic_over_algorithmic": (traffic / alg) if traffic else None,
            "alu_view": {"useful_tflops": achieved, "issued_tflops":
                         candidates * FLOP_PER_PAIR / (prof["force_ms"] * 1e-3) / 1e12,
                         "peak_tflops": FP32_VECTOR_PEAK, "frac": achieved / FP32_VECTOR_PEAK,
                         "frac_of_packed_peak": achieved / FP32_VECTOR_PEAK_PACKED,
                         "ordered_pairs_per_launch": pairs, "list_candidates_per_launch": candidates}}
    analysis = None if a.no_analysis else time_analysis(s, md, rep)
    if analysis:
        log(f"analysis: {analysis}")
    s.close()
    del s
    torch.cuda.empty_cache()

    fp64 = None
    if not a.no_fp64 and a.precision != "fp64":
        s2, _ = make_system(wl, "fp64", md)
        equilibrate(s2, md, a.equil)
        s2.set_list_params(skin, int(st["cell_div"]))
        s2.step_nve(a.warmup)
        k2 = max(100, a.steps // 2)
        el2, f0, f1 = timed_graph(s2, md, torch, k2)
        p2 = md.md_profile(s2.ctx, min(100, a.profile_steps))
        fp64 = {"value": n * k2 / el2, "steps": k2, "ms_per_step": el2 * 1e3 / k2,
                "drift_per_1e4": abs(f1 - f0) / abs(f0) * (1e4 / k2), "force_ms": p2["force_ms"]}
        log(f"fp64 GPU: {fp64}")
        s2.close()
        del s2
        torch.cuda.empty_cache()

    batch = None
    if not a.no_batch:
        batch = batched(md, torch, W, a.batch_steps)
        log(f"batched: {batch}")
        torch.cuda.empty_cache()

    planar = None
    if a.planar:
        planar = planar_leg(md, torch, W)
        log(f"planar: {planar}")
        torch.cuda.empty_cache()

    lad = None
    if a.ladder:
        lad = ladder_leg(md, W)
        log(f"ladder: {lad}")

    batch_large = None
    if a.batch_large:
        batch_large = batched_large(md, torch, W)
        log(f"batched large: {batch_large}")
        torch.cuda.empty_cache()

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(wl, a.cpu_seconds)
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": "atom-steps/s, KA LJ N=1M + batched replicas, mixed vs FP64, ≤1e-4 drift",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32/f64", "mixed_fixed": "f32/f64/i64"}[a.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "n_atoms": n, "precision": a.precision, "dt": wl.dt,
                   "skin": skin, "cell_div": int(st["cell_div"]), "init": init, "equil_steps": a.equil,
                   "hip_graph": True, "parallelism": "single-gpu"},
        "drift_per_1e4_steps": drift,
        "energy_per_atom": [e0 / n, e1 / n],
        "rebuilds_per_step": prof["rebuilds"] / prof["steps"],
        "roofline": roof,
        "fp64_gpu": fp64,
        "speedup_vs_fp64_gpu": (value / fp64["value"]) if fp64 else None,
        "batched": batch,
        "batched_large": batch_large,
        "ladder": lad,
        "planar": planar,
        "cpu_baseline": cpu,
        "autotune": tune,
        "analysis": analysis,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
