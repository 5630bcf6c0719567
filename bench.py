"""Throughput benchmark of the Kob-Andersen MD hot path on one MI355X.

Headline (`value`): N = 1,048,576 Kob-Andersen particles (838,861 A / 209,715
B) at density 1.2 and T = 0.45, dt = 0.005, mixed precision with 64-bit
fixed-point force sums.  Set-up (not timed): simple-cubic lattice with B/A
swaps, Maxwell-Boltzmann velocities, stochastic-bath equilibration,
neighbour-list autotuning, warm-up steps.  Timed: K NVE velocity-Verlet steps
replayed from a captured HIP graph (forces, integration and every list rebuild
included).  One JSON line on stdout.

Also measured, in extra keys (all inputs seeded and synthetic):
  - the energy drift of the headline system over 10^4 further NVE steps, from
    the observables the library samples on the device every 10 steps
    (500-step window means, and the least-squares slope);
  - the same system in FP64 (10^4 graph-replayed steps, with drift);
  - the roofline of the step kernel: useful FP32 FLOP (ordered in-cutoff pairs
    x 19) per launch over its mean launch time (HIP events on the context
    stream), against the FP32 vector peak; issued FLOP and an HBM view beside;
  - N = 1000 in FP64; N = 32,000 in FP64 and in mixed precision, with the
    pair-distance histogram every 100 steps and the MSD on the paper's
    log-spaced steps for four origins; the 256-replica batch with the drift of
    every replica; the 64-replica large batch admitted by footprint;
  - the FP64 CPU oracle (median of 3 runs on 1 core and on all cores).
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
FP32_PEAK = 157.3           # MI355X FP32 vector peak, TFLOP/s (published; packed FP32)
FP32_PEAK_NONPACKED = 78.6  # 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz, one FMA per lane per cycle
HBM_PEAK = 8000.0           # GB/s
# Minimal HBM bytes of one atom-step of the integration (read r, v, a; write
# r, v and the position mirror): the algorithmic figure the HBM view uses.
INTEGRATION_BYTES = 150
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kernel_hbm_traffic.md")
TRAFFIC_SOURCES = ("paper_2001_07089_amd/csrc/kernels_force.hip", "paper_2001_07089_amd/csrc/common_dev.hpp",
                   "paper_2001_07089_amd/csrc/kamd_internal.hpp")
SAMPLE_EVERY = 10
# tuned picks shipped with the package (tune_cache format, keyed by device and workload class)
TUNE_CACHE = os.path.join(ROOT, "paper_2001_07089_amd", "tuned", "autotune.json")
TUNE = {"path": TUNE_CACHE, "refresh": False}


def tuned(s, probe_steps):
    """The autotuner's pick for this system: from the cache when it holds one
    for the workload class on this device, else from md_autotune (stored)."""
    from paper_2001_07089_amd import tune_cache
    return tune_cache.tune(s, probe_steps, path=TUNE["path"], refresh=TUNE["refresh"])


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
    p.add_argument("--tune-cache", default=TUNE_CACHE,
                   help="autotuner cache: a stored pick for the workload class and device is applied as is "
                        "(reproducible list parameters, hence trajectories); a miss runs the autotuner and stores")
    p.add_argument("--retune", action="store_true", help="run the autotuner even where the cache holds a pick")
    p.add_argument("--skin", type=float, default=None, help="fixed list skin (skips the autotuner)")
    p.add_argument("--cell-div", type=int, default=1, help="cell division with --skin")
    p.add_argument("--drift-steps", type=int, default=10000, help="NVE steps of each drift measurement")
    p.add_argument("--windows", type=int, default=None, choices=[0, 1],
                   help="force the step-kernel variant (mixed precisions): 1 gathers from LDS windows of the "
                        "stencil rows, 0 from global memory (default: the autotuner's choice)")
    p.add_argument("--wg", type=int, default=None, choices=[64, 128, 256],
                   help="force the step kernel's threads per block (default: the autotuner's choice)")
    p.add_argument("--profile-steps", type=int, default=200)
    p.add_argument("--no-analysis", action="store_true", help="skip the RDF / MSD timings")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU run of the headline system")
    p.add_argument("--no-small", action="store_true", help="skip the N = 1000 FP64 leg")
    p.add_argument("--no-medium", action="store_true", help="skip the N = 32,000 leg")
    p.add_argument("--no-batch", action="store_true", help="skip the 256-replica leg")
    p.add_argument("--no-batch-large", action="store_true", help="skip the 64-replica large batch")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--only-headline", action="store_true", help="the headline and its drift only")
    p.add_argument("--only-batch", action="store_true",
                   help="the 256-replica leg only (its JSON object on one line), e.g. for a kernel trace of it")
    p.add_argument("--cpu-steps", type=int, default=3, help="oracle steps per all-core run")
    p.add_argument("--batch-drift-study", action="store_true",
                   help="also run the 256-replica batch's worst-drifting replicas in FP64 at dt 0.005 and 0.0025")
    p.add_argument("--planar", action="store_true",
                   help="also run the planar KA variant (65:35, N/L^2 = 1.204) at N = 2^20, T = 0.4")
    p.add_argument("--ladder", action="store_true",
                   help="also run a temperature ladder: 64 independent N=1000 ladders through T = 3.0 ... 0.5")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB (5 times) and exit: the reference "
                        "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    a = p.parse_args()
    TUNE["path"], TUNE["refresh"] = a.tune_cache, a.retune
    if a.only_headline:
        a.no_fp64 = a.no_small = a.no_medium = a.no_batch = a.no_batch_large = a.no_cpu = True
        a.no_analysis = True
    return a


# ------------------------------------------------------------------ helpers
def ring_rows(steps):
    return steps // SAMPLE_EVERY + 64


def make_system(md, rep, precision, dt, init, samples=0, **kw):
    return md.System([(rep.n, rep.n_a, rep.box, rep.temperature, rep.seed)], precision=precision, dt=dt, skin=0.3,
                     init=init, auto_sync=False, sample_every=SAMPLE_EVERY if samples else 0,
                     sample_capacity=ring_rows(samples) if samples else 0, **kw)


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


def timed_graph(s, torch, steps):
    """Capture `steps` NVE steps, replay once untimed, then time one replay."""
    s.capture(steps)
    s.launch()
    s.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.launch()
    s.stream.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def drift_run(s, torch, steps, chunk=1000):
    """`steps` NVE steps as replays of a captured `chunk`-step graph, sampled
    every SAMPLE_EVERY steps on the device.  Returns (seconds, rows [R][S][6])."""
    chunk = min(chunk, steps)
    s.capture(chunk)
    s.launch()                      # warm replay, not sampled for the drift
    s.stream.synchronize()
    s.clear_samples()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, steps // chunk)):
        s.launch()
    s.stream.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, s.samples(ring_rows(steps))


def drift_stats(rows, n):
    from paper_2001_07089_amd import analysis
    d = analysis.energy_drift(rows, 500)
    d["per_particle_e"] = d.pop("e_mean") / n
    return d


def kernel_name(precision, windows=0, wg=256):
    """The step kernel of NVE steps (forces fused with the closing half kick
    and the next drift), with its template arguments: FIXED, ENERGY, KD,
    then STAGE and waves per block for the mixed precisions."""
    if precision == "fp64":
        return f"k_force_fp64<false,true,{wg // 64}>"
    fixed = "true" if precision == "mixed_fixed" else "false"
    return f"k_force_mixed<{fixed},false,true,{'true' if windows else 'false'},{wg // 64}>"


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_records(path=None):
    """The machine-readable records of the committed counter summary: one
    dict per "### Record" section of "- key: value" lines."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return []
    recs, cur = [], None
    for line in text.splitlines():
        if line.startswith("### Record"):
            cur = {}
            recs.append(cur)
        elif cur is not None and line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            cur[k.strip()] = v.strip().strip("`")
    return recs


def stored_traffic(skin, cell_div, precision, n, kernel):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, when a record there was taken on the current kernel source at the
    same list parameters, precision, size and kernel variant; otherwise None."""
    digest = source_digest()
    for kv in traffic_records():
        try:
            ok = (kv["source_digest"] == digest and abs(float(kv["skin"]) - skin) < 1e-9
                  and int(kv["cell_div"]) == cell_div and kv["precision"] == precision
                  and int(kv["n_atoms"]) == n and kv.get("kernel") == kernel)
            if ok:
                return float(kv["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def roofline(prof, stats, n, precision):
    """The step kernel priced against the FP32 vector peak.  Work unit: the
    ordered in-cutoff pair (the list is full, so each unordered pair is
    evaluated from both sides, as Eq. (KAFix) sums over all partners j),
    19 FLOP each; units per launch from a closing energy pass (md_profile);
    the launch time is the mean of HIP events around every step-kernel launch
    on the context stream."""
    sec = prof["force_ms"] * 1e-3
    pairs = prof["pairs"]
    useful = pairs * FLOP_PER_PAIR / sec / 1e12
    candidates = stats["mean_list_len"] * n
    walked = stats.get("mean_walked", stats["mean_list_len"]) * n  # padded to each wavefront's longest
    kname = kernel_name(precision, int(stats["windows"]), int(stats["wg_size"]))
    traffic = stored_traffic(stats["skin"], int(stats["cell_div"]), precision, n, kname)
    alg_bytes = n * INTEGRATION_BYTES
    return {"bound": "alu", "achieved": useful, "peak": FP32_PEAK, "unit": "TFLOP/s", "frac": useful / FP32_PEAK,
            "traffic": traffic, "kernel": kname, "kernel_ms": prof["force_ms"],
            "work_unit": "ordered in-cutoff pair", "flop_per_unit": FLOP_PER_PAIR, "units_per_launch": pairs,
            "frac_of_nonpacked_peak": useful / FP32_PEAK_NONPACKED,
            "issued_tflops": walked * FLOP_PER_PAIR / sec / 1e12, "list_candidates_per_launch": candidates,
            "walked_entries_per_launch": walked,
            "hbm_view": {"algorithmic_bytes_per_launch": alg_bytes, "bytes_per_atom_step": INTEGRATION_BYTES,
                         "achieved_gbs": alg_bytes / sec / 1e9, "peak_gbs": HBM_PEAK,
                         "frac": alg_bytes / sec / 1e9 / HBM_PEAK,
                         "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None}}


def rdf_first_peaks(s, rep, hist=None):
    """g_AA, g_AB, g_BB (Eqs. (gAA), (gAB)) of one on-device RDF sample (r_max
    5.0, 200 bins), host-normalised: (r, g) of each first peak, so that runs
    in different precisions can be set side by side."""
    from paper_2001_07089_amd import analysis
    dr = 5.0 / 200
    h = s._host(s.rdf(dr, 200) if hist is None else hist)[0]
    r, g = analysis.rdf(h, rep.n, rep.n_a, rep.box, dr)
    m = r < 1.5
    out = {}
    for k, name in enumerate(("AA", "AB", "BB")):
        i = int(np.argmax(g[k][m]))
        out[name] = [float(r[m][i]), float(g[k][m][i])]
    return out


def time_analysis(s, rep):
    """On-device RDF (r_max 5.0, 200 bins) and MSD (one origin, one
    measurement) of the large system, each timed on its own."""
    import torch
    from paper_2001_07089_amd import analysis
    dr = 5.0 / 200
    s.rdf(dr, 200)
    s.stream.synchronize()
    t0 = time.perf_counter()
    h = s.rdf(dr, 200)
    s.stream.synchronize()
    t_rdf = time.perf_counter() - t0
    counts = s._host(h).astype(np.int64)[0].sum(axis=1)
    peaks = rdf_first_peaks(s, rep, h)
    # the LAMMPS compute rdf layout: 25 bins to the force cutoff 2.5, with
    # coordination numbers (host normalisation of the device counts)
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
            "rdf_pair_counts_AA_AB_BB": [int(c) for c in counts], "rdf_first_peaks_r_g": peaks,
            "lammps_rdf_ms": t_lmp * 1e3, "lammps_rdf_coordination_at_2.5_AA_BB_AB":
                [float(table[-1, 3]), float(table[-1, 5]), float(table[-1, 7])],
            "msd_ms": t_msd * 1e3, "msd_after_100_steps_A_B": [float(m[0, 0]), float(m[0, 1])]}


# --------------------------------------------------------------------- legs
def fp64_leg(md, torch, wl, init, equil, warmup, skin, cell_div, steps, profile_steps):
    """The headline system in FP64 ("plain"): same start, bath and list
    parameters; 10^4 NVE steps from graph replays, with drift."""
    rep = wl.replicas[0]
    s = make_system(md, rep, "fp64", wl.dt, init, samples=steps)
    equilibrate(s, md, equil)
    s.set_list_params(skin, cell_div)
    s.step_nve(warmup)
    el, rows = drift_run(s, torch, steps)
    peaks = rdf_first_peaks(s, rep)
    prof = md.md_profile(s.ctx, min(100, profile_steps))
    out = {"value": rep.n * steps / el, "unit": "atom-steps/s", "steps": steps, "ms_per_step": el * 1e3 / steps,
           "drift": drift_stats(rows[0], rep.n), "rdf_first_peaks_r_g": peaks, "force_ms": prof["force_ms"],
           "device_error_word": s.status()}
    s.close()
    return out


def small_leg(md, torch, W, steps=1000):
    """N = 1000 (800 A / 200 B), density 1.2, T0 = 2.0, FP64 throughout: RSA
    start with Maxwell-Boltzmann velocities, 100 NVE steps in which the random
    start relaxes, then `steps` NVE steps from a graph replay with drift."""
    wl = W.ka_small()
    rep = wl.replicas[0]
    s = make_system(md, rep, "fp64", wl.dt, "rsa", samples=steps)
    s.step_nve(100)
    el, rows = drift_run(s, torch, steps, chunk=steps)
    out = {"workload": wl.name, "n_atoms": rep.n, "precision": "fp64", "steps": steps,
           "value": rep.n * steps / el, "unit": "atom-steps/s", "ms_per_step": el * 1e3 / steps,
           "drift": drift_stats(rows[0], rep.n), "device_error_word": s.status()}
    s.close()
    return out


def medium_leg(md, torch, W, nvt_steps=20000, nve_steps=10000):
    """N = 32,000 at density 1.2: stochastic bath at T = 0.5 for 2*10^4 steps
    (redraw every 50 after 500 steps every 10), then from that one state
    10^4 NVE steps in FP64 and in mixed precision (graph replays, drift).
    Analysis run (mixed, eager segments): RDF 200 bins to L/2 every 100
    steps; MSD on the log-spaced steps of Sec. VI.B.1 (t0 = 1, kmax = 60) for
    origins at steps 0, 10, 100 and 500; each sample timed on its own."""
    from paper_2001_07089_amd import analysis
    wl = W.ka_medium()
    rep = wl.replicas[0]
    t0 = time.perf_counter()
    s = make_system(md, rep, "mixed_fixed", wl.dt, "rsa")
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(nvt_steps - 500, md.NVT_STOCHASTIC, n_reassign=50)
    s.sync()
    st = s.numpy(("x", "y", "z", "vx", "vy", "vz"))
    s.close()
    t_nvt = time.perf_counter() - t0
    out = {"workload": wl.name, "n_atoms": rep.n, "nvt_steps": nvt_steps, "nve_steps": nve_steps,
           "nvt_seconds": t_nvt}
    for prec in ("fp64", "mixed"):
        c = md.System([(rep.n, rep.n_a, rep.box, rep.temperature, rep.seed)], precision=prec, dt=wl.dt, skin=0.3,
                      positions=(st["x"], st["y"], st["z"]), velocities=(st["vx"], st["vy"], st["vz"]),
                      auto_sync=False, sample_every=SAMPLE_EVERY, sample_capacity=ring_rows(nve_steps))
        el, rows = drift_run(c, torch, nve_steps)
        out[prec] = {"value": rep.n * nve_steps / el, "unit": "atom-steps/s", "ms_per_step": el * 1e3 / nve_steps,
                     "drift": drift_stats(rows[0], rep.n), "T_mean": float(rows[0][:, 4].mean()),
                     "device_error_word": c.status()}
        c.close()
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    # analysis run
    c = md.System([(rep.n, rep.n_a, rep.box, rep.temperature, rep.seed)], precision="mixed", dt=wl.dt, skin=0.3,
                  positions=(st["x"], st["y"], st["z"]), velocities=(st["vx"], st["vy"], st["vz"]), auto_sync=False)
    origins = [0, 10, 100, 500]
    sched = {k: [t0_ + int(t) for t in md.md_log_schedule(nve_steps - t0_)] for k, t0_ in enumerate(origins)}
    events = {}
    for k, t0_ in enumerate(origins):
        events.setdefault(t0_, []).append(("origin", k))
        for t in sched[k]:
            events.setdefault(t, []).append(("msd", k))
    for t in range(100, nve_steps + 1, 100):
        events.setdefault(t, []).append(("rdf", 0))
    dr, nb = 0.5 * rep.box / 200, 200
    hist = c._zeros((1, 3, nb), c.torch.int64)
    msd = {k: [] for k in range(len(origins))}
    t_rdf = t_msd = 0.0
    n_rdf = n_msd = 0
    cur = 0
    for t in sorted(events):
        if t > cur:
            c.step_nve(t - cur)
            cur = t
        c.stream.synchronize()
        for kind, k in events[t]:
            t1 = time.perf_counter()
            if kind == "origin":
                c.msd_set_origin(k)
            elif kind == "msd":
                msd[k].append((t - origins[k], c.msd(k)[0].tolist()))
                t_msd += time.perf_counter() - t1
                n_msd += 1
            else:
                c.rdf(dr, nb, hist)
                c.stream.synchronize()
                t_rdf += time.perf_counter() - t1
                n_rdf += 1
    r, g = analysis.rdf(c._host(hist)[0], rep.n, rep.n_a, rep.box, dr, n_rdf)
    ipk = int(np.argmax(g[0]))
    last = {k: v[-1] for k, v in msd.items()}
    out["analysis"] = {"rdf_samples": n_rdf, "rdf_ms_per_sample": t_rdf * 1e3 / max(n_rdf, 1),
                       "rdf_bins": nb, "rdf_r_max": nb * dr, "g_AA_first_peak": [float(r[ipk]), float(g[0, ipk])],
                       "g_AA_mean_beyond_6": float(g[0][r > 6.0].mean()),
                       "msd_measurements": n_msd, "msd_ms_per_measurement": t_msd * 1e3 / max(n_msd, 1),
                       "msd_lags_per_origin": {str(o): len(msd[k]) for k, o in enumerate(origins)},
                       "msd_A_B_at_last_lag": {str(o): last[k] for k, o in enumerate(origins)},
                       "device_error_word": c.status()}
    c.close()
    return out


def batched(md, torch, W, steps):
    """256 replicas, N uniform on [250, 8000], T on [0.45, 2.0], mixed precision:
    one launch per kernel per step over all replicas, graph replays; the drift
    of every replica over `steps` NVE steps."""
    wl = W.ka_batch_small()
    reps = [(r.n, r.n_a, r.box, r.temperature, r.seed) for r in wl.replicas]
    t0 = time.perf_counter()
    s = md.System(reps, precision="mixed", dt=wl.dt, skin=0.3, init="rsa", auto_sync=False,
                  sample_every=SAMPLE_EVERY, sample_capacity=ring_rows(steps))
    log(f"batch init (rsa, {len(reps)} replicas, {wl.n_total} particles) {time.perf_counter() - t0:.1f} s")
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(1500, md.NVT_STOCHASTIC, n_reassign=50)
    tune = tuned(s, 60)
    s.step_nve(200)
    el, rows = drift_run(s, torch, steps)
    from paper_2001_07089_amd import analysis
    d = np.array([analysis.energy_drift(rows[k], 500)["windowed"] for k in range(len(reps))])
    sl = np.array([analysis.energy_drift(rows[k], 500)["slope"] for k in range(len(reps))])
    worst = [int(k) for k in np.argsort(-d)[:8]]
    out = {"workload": wl.name, "n_replicas": len(reps), "n_atoms": wl.n_total, "precision": "mixed",
           "steps": steps, "value": wl.n_total * steps / el, "unit": "atom-steps/s",
           "ms_per_step": el * 1e3 / steps, "drift_windowed_median": float(np.median(d)),
           "drift_windowed_max": float(d.max()), "drift_slope_median": float(np.median(sl)),
           "replicas_above_1e-4": int((d > 1e-4).sum()),
           "worst": [{"replica": k, "n": reps[k][0], "T": reps[k][3], "drift": float(d[k])} for k in worst],
           "autotune": tune, "device_error_word": s.status()}
    s.close()
    return out


def batch_drift_study(md, torch, W, worst, steps=10000):
    """The batch's worst-drifting replicas alone in FP64 at dt = 0.005 and at
    dt = 0.0025 (the same physical time: twice the steps): whether the drift
    is the time step's or the precision's."""
    from paper_2001_07089_amd import analysis
    wl = W.ka_batch_small()
    out = []
    for w in worst[:4]:
        r = wl.replicas[w["replica"]]
        row = {"replica": w["replica"], "n": r.n, "T": r.temperature, "mixed_dt0.005": w["drift"]}
        for dt in (0.005, 0.0025):
            n = int(round(steps * 0.005 / dt))
            s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="fp64", dt=dt, skin=0.3,
                          init="rsa", auto_sync=False, sample_every=SAMPLE_EVERY, sample_capacity=ring_rows(n))
            s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
            s.step_nvt(1500, md.NVT_STOCHASTIC, n_reassign=50)
            s.step_nve(200)
            _, rows = drift_run(s, torch, n)
            dd = analysis.energy_drift(rows[0], int(500 * 0.005 / dt))
            row[f"fp64_dt{dt}"] = dd["windowed"] * (n / steps)  # per the same physical time as 10^4 steps at 0.005
            s.close()
        out.append(row)
    return out


def batched_large(md, torch, W):
    """64 replicas, N uniform on [5e4, 5e5], density in {1.1, 1.2, 1.3}, T on
    [0.45, 1.0], MIXED: admission against the free device memory, lattice
    start, 1000 stochastic-bath steps, then 1000 NVE steps replayed from a
    graph in four blocks of 250 with an RDF sample (r_max 5.0, 200 bins) and
    an MSD origin at the start of each block.  The NVE steps are timed; the
    RDF and MSD calls are timed on their own."""
    from paper_2001_07089_amd import analysis
    wl = W.ka_batch_large()
    reps_all = md.make_replicas([(r.n, r.n_a, r.box, r.temperature, r.seed) for r in wl.replicas])
    cfg = md.make_config("mixed", wl.dt, 0.3, md.INIT_LATTICE, sample_every=SAMPLE_EVERY,
                         sample_capacity=ring_rows(1000), msd_slots=4)
    free, _ = torch.cuda.mem_get_info()
    adm, cnt = md.md_admit(cfg, reps_all, int(free * 0.8))
    chosen = [r for r, a in zip(wl.replicas, adm) if a]
    reps = [(r.n, r.n_a, r.box, r.temperature, r.seed) for r in chosen]
    n_tot = sum(r.n for r in chosen)
    t0 = time.perf_counter()
    s = md.System(reps, precision="mixed", dt=wl.dt, skin=0.3, init="lattice", auto_sync=False,
                  sample_every=SAMPLE_EVERY, sample_capacity=ring_rows(1000), msd_slots=4)
    log(f"batch-large init ({cnt} of {len(wl.replicas)} replicas admitted, {n_tot} particles) "
        f"{time.perf_counter() - t0:.1f} s")
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=10)
    s.step_nvt(500, md.NVT_STOCHASTIC, n_reassign=50)
    dr = 5.0 / 200
    s.capture(250)
    s.clear_samples()
    t_nve = t_rdf = 0.0
    hist = s._zeros((len(reps), 3, 200), s.torch.int64)
    for blk in range(4):
        t1 = time.perf_counter()
        s.msd_set_origin(blk)
        s.rdf(dr, 200, hist)
        s.stream.synchronize()
        t_rdf += time.perf_counter() - t1
        t1 = time.perf_counter()
        s.launch()
        s.stream.synchronize()
        t_nve += time.perf_counter() - t1
    t1 = time.perf_counter()
    msd = [s.msd(k) for k in range(4)]
    t_msd = time.perf_counter() - t1
    rows = s.samples(ring_rows(1000))
    d = np.array([analysis.energy_drift(rows[k], 500)["windowed"] for k in range(len(reps))])
    out = {"workload": wl.name, "n_replicas_admitted": cnt, "n_replicas": len(wl.replicas), "n_atoms": n_tot,
           "precision": "mixed", "nve_steps": 1000, "value": n_tot * 1000 / t_nve, "unit": "atom-steps/s",
           "ms_per_step": t_nve * 1e3 / 1000, "rdf_ms_per_sample": t_rdf * 1e3 / 4,
           "msd_ms_per_measurement": t_msd * 1e3 / 4, "drift_windowed_median": float(np.median(d)),
           "drift_windowed_max": float(d.max()), "drift_note": "1000 NVE steps: two 500-step windows",
           "msd_A_after_1000_steps_median": float(np.median(msd[0][:, 0])),
           "workspace_bytes": int(s.ws_bytes), "device_error_word": s.status()}
    s.close()
    return out


def planar_leg(md, torch, W, steps=1000):
    """The planar KA variant of the appendix exercise at N = 2^20: square
    lattice start, 12,000 bath steps at T = 0.4 with a redraw every 10 steps,
    then graph-replayed NVE steps timed (and their drift)."""
    wl = W.ka_planar(1 << 20, 0.4)
    r = wl.replicas[0]
    s = md.System([(r.n, r.n_a, r.box, r.temperature, r.seed)], precision="mixed_fixed", dt=wl.dt, skin=0.3,
                  init="lattice", auto_sync=False, dim=2, sample_every=SAMPLE_EVERY,
                  sample_capacity=ring_rows(10000))
    s.step_nvt(12000, md.NVT_STOCHASTIC, n_reassign=10)
    tune = tuned(s, 100)
    s.step_nve(200)
    el = timed_graph(s, torch, steps)
    _, rows = drift_run(s, torch, 10000)
    out = {"workload": wl.name, "n_atoms": r.n, "box": r.box, "value": r.n * steps / el, "unit": "atom-steps/s",
           "ms_per_step": el * 1e3 / steps, "drift": drift_stats(rows[0], r.n), "bath_steps": 12000,
           "T_after": float(rows[0][-1, 4]), "autotune": tune, "device_error_word": s.status()}
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, steps_all=3, steps_one=1):
    """The FP64 oracle (cell list, OpenMP) on the host cores: median of 3 runs
    of `steps_all` velocity-Verlet steps on all cores and of `steps_one` on
    one core, on the headline system's size and density (a jittered lattice,
    the workload's own start; pair counts per particle as in the liquid)."""
    import oracle as O
    from paper_2001_07089_amd import workload as W
    rep = wl.replicas[0]
    x, y, z = W.lattice_config(rep.n, rep.box, rep.seed, 0.1)
    vx, vy, vz = W.gaussian_velocities(rep.n, math.sqrt(rep.temperature), rep.seed + 1)
    O.set_num_threads(0)
    n_all = O.num_threads()
    st = O.State(x, y, z, vx, vy, vz, rep.n_a, rep.box)
    st.compute_forces("cell")

    def runs(k):
        rates = []
        for _ in range(3):
            t0 = time.perf_counter()
            O.run(st, wl.dt, k, method="cell")
            rates.append(rep.n * k / (time.perf_counter() - t0))
        return float(np.median(rates)), rates

    v_all, r_all = runs(steps_all)
    O.set_num_threads(1)
    v_one, r_one = runs(steps_one)
    O.set_num_threads(0)
    return {"value": v_all, "unit": "atom-steps/s", "cores": n_all, "kind": "oracle",
            "sample": f"median of 3 runs of {steps_all} velocity-Verlet NVE steps of the same N={rep.n} "
                      f"system (cell-list oracle, FP64, OpenMP on {n_all} threads)",
            "runs": r_all, "one_core": {"value": v_one, "cores": 1, "runs": r_one,
                                        "sample": f"median of 3 runs of {steps_one} step(s) on one thread"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


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

    if a.only_batch:
        t1 = time.perf_counter()
        out = batched(md, torch, W, a.drift_steps)
        log(f"batched ({time.perf_counter() - t1:.1f} s): {out}")
        print(json.dumps(out), flush=True)
        return

    wl = {"small": W.ka_small, "medium": W.ka_medium, "large": W.ka_large}[a.workload]()
    rep = wl.replicas[0]
    n = rep.n
    init = "rsa" if n <= 300000 else "lattice"
    log(f"workload {wl.name}: N={n} L={rep.box:.6f} T={rep.temperature} precision={a.precision}")

    t0 = time.perf_counter()
    s = make_system(md, rep, a.precision, wl.dt, init, samples=a.drift_steps)
    log(f"init ({init}) {time.perf_counter() - t0:.1f} s")
    # melt the start, tune the list on the liquid, then equilibrate at the
    # tuned list parameters (so nearly every launch of the run, and of a
    # kernel trace of it, uses them)
    first = min(1000, a.equil)
    equilibrate(s, md, first)
    tune = None
    if a.skin is not None:
        s.set_list_params(a.skin, a.cell_div)
        log(f"list parameters fixed: skin {a.skin}, cell_div {a.cell_div}")
    elif not a.no_autotune:
        tune = tuned(s, 100)
        log(f"autotune: {tune}")
    if a.windows is not None or a.wg is not None:
        st0 = md.md_stats(s.ctx)
        win = a.windows if a.windows is not None else int(st0["windows"])
        s.set_force_kernel(win, a.wg or 0)
        log(f"step kernel fixed: windows {win}, threads per block {a.wg or int(st0['wg_size'])}")
    if a.equil > first:
        s.step_nvt(a.equil - first, md.NVT_STOCHASTIC, n_reassign=50)
    log(f"equilibrated {a.equil} steps, {time.perf_counter() - t0:.1f} s")
    s.step_nve(a.warmup)
    s.stream.synchronize()
    el = timed_graph(s, torch, a.steps)
    value = n * a.steps / el
    log(f"timed {a.steps} steps: {el * 1e3:.2f} ms -> {value:.4e} atom-steps/s")
    el_d, rows = drift_run(s, torch, a.drift_steps)
    drift = drift_stats(rows[0], n)
    log(f"drift over {a.drift_steps} NVE steps: {drift}, {n * a.drift_steps / el_d:.4e} atom-steps/s")
    prof = md.md_profile(s.ctx, a.profile_steps)
    st = md.md_stats(s.ctx)
    w = s.status()
    log(f"profile: {prof}")
    log(f"stats: {st}  err=0x{w:x}")
    roof = roofline(prof, st, n, a.precision)
    analysis_out = None if a.no_analysis else time_analysis(s, rep)
    if analysis_out:
        log(f"analysis: {analysis_out}")
    s.close()
    del s
    torch.cuda.empty_cache()

    legs = {}

    def leg(name, fn, *args):
        t1 = time.perf_counter()
        try:
            legs[name] = fn(*args)
        finally:
            torch.cuda.empty_cache()
        log(f"{name} ({time.perf_counter() - t1:.1f} s): {legs[name]}")

    if not a.no_fp64 and a.precision != "fp64":
        leg("fp64_gpu", fp64_leg, md, torch, wl, init, a.equil, a.warmup, st["skin"], int(st["cell_div"]),
            a.drift_steps, a.profile_steps)
    if not a.no_small:
        leg("small_n1000_fp64", small_leg, md, torch, W)
    if not a.no_medium:
        leg("medium_n32000", medium_leg, md, torch, W)
    if not a.no_batch:
        leg("batched", batched, md, torch, W, a.drift_steps)
        if a.batch_drift_study:
            leg("batch_drift_study", batch_drift_study, md, torch, W, legs["batched"]["worst"])
    if not a.no_batch_large:
        leg("batched_large", batched_large, md, torch, W)
    if a.planar:
        leg("planar", planar_leg, md, torch, W)
    if a.ladder:
        leg("ladder", ladder_leg, md, W)
    cpu = None
    if not a.no_cpu:
        t1 = time.perf_counter()
        cpu = cpu_baseline(wl, a.cpu_steps)
        log(f"cpu oracle ({time.perf_counter() - t1:.1f} s): {cpu}")

    fp64 = legs.get("fp64_gpu")
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
                   "skin": st["skin"], "cell_div": int(st["cell_div"]), "step_kernel_windows": int(st["windows"]),
                   "step_kernel_threads_per_block": int(st["wg_size"]), "init": init, "equil_steps": a.equil,
                   "hip_graph": True, "parallelism": "single-gpu"},
        "drift": dict(drift, nve_steps=a.drift_steps, atom_steps_per_s=n * a.drift_steps / el_d),
        "rebuilds_per_step": prof["rebuilds"] / prof["steps"],
        "roofline": roof,
        "fp64_gpu": fp64,
        "speedup_vs_fp64_gpu": (value / fp64["value"]) if fp64 else None,
        "small_n1000_fp64": legs.get("small_n1000_fp64"),
        "medium_n32000": legs.get("medium_n32000"),
        "batched": legs.get("batched"),
        "batch_drift_study": legs.get("batch_drift_study"),
        "batched_large": legs.get("batched_large"),
        "planar": legs.get("planar"),
        "ladder": legs.get("ladder"),
        "cpu_baseline": cpu,
        "autotune": tune,
        "analysis": analysis_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
