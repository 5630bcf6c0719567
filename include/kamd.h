/*
 * kamd.h -- C ABI of the MI355X (gfx950) Kob-Andersen binary Lennard-Jones
 * molecular-dynamics library.
 *
 * Method: "Introduction to molecular dynamics simulations", K. Vollmayr-Lee,
 * arXiv:2001.07089.  The library advances one or many independent systems
 * ("replicas") of the Kob-Andersen 80:20 mixture (Sec. II.B) in cubic periodic
 * boxes (Sec. II.C) with velocity Verlet (Sec. II.D), the stochastic bath
 * (Sec. II.E.1, Sec. III.G) or Nose-Hoover via Fox-Andersen (Appendix B), and
 * measures the radial distribution function (Sec. VI.A) and the mean-square
 * displacement (Sec. VI.B) on the device.
 *
 * General rules
 *   - Every function returns an int: KAMD_OK (0) or a negative error code.
 *     Functions never throw, exit or print; md_last_error() gives a message.
 *   - Device pointers are plain HIP device addresses (for example the
 *     data_ptr() of a torch CUDA tensor); host pointers are ordinary memory.
 *     Which is which is stated per argument.
 *   - Arrays described as "caller order" are indexed by the caller's particle
 *     index: replica r occupies [offset_r, offset_r + n_r), its A particles
 *     first (the paper stores the A block before the B block, Sec. III.A).
 *     Particle type is implied by that position; masses are 1 (Sec. II.B).
 *   - All work is enqueued on the caller's HIP stream given to md_init and
 *     returns without waiting, except where a function is marked "syncs".
 *   - Device memory: a context works in one workspace, a block of device
 *     memory whose size md_workspace_size gives.  The caller may own it (for
 *     example a torch uint8 tensor) and pass it to md_init; the library then
 *     only borrows it and never frees it.  Given none, the library allocates
 *     it and frees it in md_destroy.  Every other buffer (state arrays,
 *     histograms, outputs) is the caller's and only borrowed.
 *   - One context must not be used from two host threads at once.
 */
#ifndef KAMD_H
#define KAMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
    KAMD_OK = 0,
    KAMD_EINVAL = -1,  /* invalid argument                                  */
    KAMD_ENOMEM = -2,  /* device memory or the admission budget is exceeded */
    KAMD_EHIP = -3,    /* a HIP runtime call failed (no device, ...)        */
    KAMD_EDEVICE = -4, /* the sticky device error word is set (md_status)   */
    KAMD_EBOX = -5,    /* box too small: largest cutoff + skin >= L/2       */
    KAMD_ESTATE = -6   /* call not valid in the current state               */
};

/* Arithmetic of the pair-force kernels. */
enum {
    KAMD_PREC_FP64 = 0,        /* binary64 throughout                                  */
    KAMD_PREC_MIXED = 1,       /* FP32 pair distances, LJ terms and pair forces from an
                                  exact fixed-point separation; FP32 per-particle partial
                                  sums converted to FP64; FP64 integration + reductions  */
    KAMD_PREC_MIXED_FIXED = 2  /* as MIXED, but every pair force is rounded to a 64-bit
                                  fixed-point integer (2^-26 units) and summed exactly:
                                  the force is independent of summation order            */
};

/* md_forces flags. */
enum { KAMD_F_FORCE = 1, KAMD_F_ENERGY = 2, KAMD_F_VIRIAL = 4 };

/* Thermostats for md_step_nvt. */
enum { KAMD_NVT_STOCHASTIC = 0, KAMD_NVT_NOSE_HOOVER = 1 };

/* Initial positions for md_init. */
enum {
    KAMD_INIT_GIVEN = 0,   /* positions and velocities are read from the caller arrays   */
    KAMD_INIT_RSA = 1,     /* random sequential addition with a minimum pair distance,
                              then Maxwell-Boltzmann velocities                           */
    KAMD_INIT_LATTICE = 2  /* simple cubic lattice with B/A swaps (Sec. III.A), then
                              Maxwell-Boltzmann velocities                                */
};

/* Bits of the sticky device error word (md_status). */
enum {
    KAMD_DEV_NONFINITE = 1u,     /* a position, velocity or force became inf/nan       */
    KAMD_DEV_LIST_OVERFLOW = 2u, /* a neighbour list exceeded its capacity            */
    KAMD_DEV_FORCE_RANGE = 4u,   /* MIXED_FIXED: a pair came so close that its force
                                    reached 2^25 (beyond it the 2^-26-unit rounding is
                                    no longer exact), or a net force exceeded 1e8     */
    KAMD_DEV_LIST_FORMAT = 8u,   /* internal: a force kernel met a list part stored in
                                    a format it does not read, and skipped it          */
    KAMD_DEV_RUNAWAY = 16u       /* a particle moved more than half the smallest sigma
                                    in one step (a normal step moves about a hundredth
                                    of that): forces too large for the time step, as
                                    the close pairs of a random start give (the runaway
                                    positions and velocities of Sec. II.F).  The lists
                                    stay valid (they are checked every step); the
                                    trajectory is not to be trusted                    */
};

/* Pair model: epsilon and sigma per pair type in the order AA, AB, BB, and the
 * cutoff factor (r_c = rc_factor * sigma).  Kob-Andersen values, Sec. II.B:
 * eps = {1, 1.5, 0.5}, sigma = {1, 0.8, 0.88}, rc_factor = 2.5. */
typedef struct {
    double eps[3];
    double sigma[3];
    double rc_factor;
} kamd_model;

/* One replica: n particles of which the first n_a are type A, in a cubic box
 * of edge `box`, at bath temperature `temperature` (k_B = 1), with its own
 * random seed.  `offset` is its first index in the caller-order arrays. */
typedef struct {
    int64_t offset;
    int32_t n;
    int32_t n_a;
    double box;
    double temperature;
    uint64_t seed;
} kamd_replica;

/* Caller-order state arrays (device pointers, FP64, length n_total = sum of
 * n).  img holds the periodic image counters as three blocks of n_total int32
 * (x, y, z): the unwrapped position is x + img*L (Sec. VI.B.1).  Any pointer
 * may be NULL when the caller does not want that array exported. */
typedef struct {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *ax, *ay, *az;
    int32_t *img;
} kamd_state;

/* Run configuration. */
typedef struct {
    kamd_model model;
    int32_t precision;      /* KAMD_PREC_*                                          */
    double dt;              /* time step (LJ units)                                 */
    double skin;            /* neighbour-list skin; < 0 selects 0.3                 */
    int32_t init_mode;      /* KAMD_INIT_*                                          */
    double min_dist;        /* minimum pair distance of KAMD_INIT_RSA (e.g. 0.8)    */
    int32_t cell_div;       /* list cells per list radius: 1 or 2 (0 = 1)           */
    double list_capacity;   /* neighbour-list rows as a multiple of the expected
                               count (0 = 1.6)                                      */
    int32_t auto_sync;      /* 1: export state to the caller arrays after every call */
    int32_t dim;            /* 3 (or 0): three-dimensional; 2: the planar system of
                               the appendix exercise, every z, vz and az is 0, the
                               box is L x L at number density N/L^2, the bath and
                               temperature use 2N degrees of freedom, pressure
                               uses the area                                      */
    int32_t pe_unshifted;   /* 0: potential energy of the truncated and shifted
                               potential, Eq. (VshiftedKALJ) (the paper's Python
                               programs); 1: without the shift V_ab(r_c), the
                               energy LAMMPS pair style lj/cut reports (Sec. IV.B).
                               Forces are the same either way; only PE, E_tot and
                               everything derived from them change               */
    int32_t sample_every;   /* > 0: record the observables of every replica at the
                               end of every step whose number is a multiple of
                               this (after any thermostat action of that step)
                               into a device ring buffer read by md_observables;
                               0: no sampling.  Works inside captured graphs     */
    int32_t sample_capacity;/* rows of the ring buffer per replica (0 = 1024); the
                               oldest rows are overwritten                        */
    int32_t msd_slots;      /* MSD origin slots (0 = 16); each holds 24 bytes per
                               particle of the workspace                          */
} kamd_config;

/* Bytes of device workspace a context of this configuration needs (host
 * call, no device needed): the state and its scratch, tables, reductions,
 * observables ring, MSD origins, RDF scratch and staging, then the cell
 * arrays and the neighbour list at cfg's skin, cell division and list
 * capacity.  Exactly the layout md_init carves.  Used for admission to HBM. */
int md_workspace_size(const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
                      size_t *bytes);

/* Admission by memory footprint: walks the replicas in order and marks each
 * admitted[r] = 1 while the running footprint stays within budget_bytes,
 * else 0.  Host call.  *n_admitted receives the count. */
int md_admit(const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
             size_t budget_bytes, int32_t *admitted, int32_t *n_admitted);

typedef struct kamd_ctx kamd_ctx;

/* Create a context on the current HIP device and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  workspace: device memory of
 * ws_bytes >= md_workspace_size bytes, 256-byte aligned, owned by the caller
 * and used by nothing else while the context lives (KAMD_ENOMEM when too
 * small); NULL: the library allocates its own.  reps[] describes n_rep
 * replicas (host memory, copied).  st gives the caller-order device arrays: with
 * KAMD_INIT_GIVEN, x/y/z (in [0, L) per replica) and vx/vy/vz are read; with
 * the other init modes they are generated (RSA/lattice on the host from the
 * replica seed, velocities by the Maxwell-Boltzmann flow chart of Sec. II.E.1
 * at the replica temperature) and written to st.  Initial forces are computed
 * (the "Initialization" box of the flow chart in Sec. II.D) and written to
 * st->ax.. when given.  Errors: KAMD_EINVAL (bad sizes, n_a outside [0, n],
 * mass-free model), KAMD_EBOX (largest cutoff >= L/2), KAMD_ENOMEM,
 * KAMD_EHIP.  On error *out is NULL. */
int md_init(kamd_ctx **out, const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
            const kamd_state *st, void *workspace, size_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): md_init with the
 * workspace taken from a fixed 64 MiB device array that the library holds
 * per GPU until the process ends (about 43,000 particles with the default
 * 16 MSD origin slots, more with fewer).  Allocates no
 * device memory and calls no allocating routine.  KAMD_ENOMEM when
 * md_workspace_size exceeds 64 MiB; KAMD_ESTATE while another context works
 * in the current device's array (one at a time: two would overwrite each
 * other; md_destroy releases it).  A list that outgrows the array later is
 * reported as by a caller-owned workspace (KAMD_ENOMEM).  Everything else is
 * md_init's. */
int md_init_static(kamd_ctx **out, const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
                   const kamd_state *st, void *hip_stream);

/* Workspace the context needs now (host memory *bytes): more than it has
 * after a refused md_set_list_params or md_autotune, or after a neighbour
 * list outgrew its rows in a caller-owned workspace (those calls return
 * KAMD_ENOMEM).  No device work. */
int md_workspace_needed(kamd_ctx *ctx, size_t *bytes);

/* Move the context into another caller-owned workspace (device, ws_bytes >=
 * md_workspace_needed, 256-byte aligned, not the current one): the contents
 * are copied, the old block is no longer used (freed when it was the
 * library's own; released for another context when it was the static array
 * of md_init_static), and a captured graph is dropped (recapture).  Then repeat
 * the call that was refused.  Syncs. */
int md_set_workspace(kamd_ctx *ctx, void *workspace, size_t ws_bytes);

/* Rebuild the cell lists and neighbour lists of every replica now: bin by
 * cell, stable counting sort of the internal particle order, pair list of all
 * partners within r_c(ab) + skin (the neighbour list of Sec. III.E; LAMMPS'
 * "bin" build, Sec. IV).  Rebuilds also happen automatically inside the step
 * functions whenever a particle has moved more than skin/2 since the last
 * build.
 *
 * List overflow heals itself: a list that outgrows its rows sets
 * KAMD_DEV_LIST_OVERFLOW on the device.  md_build_cells, md_forces,
 * md_step_nve, md_step_nvt, md_import and md_set_state check for it before
 * they return; the list then grows to the rows its build asked for (plus a
 * quarter) and the call's work is redone (steps from the state the call
 * started from), so those calls sync.  In a caller-owned workspace that is
 * too small for the longer list they return KAMD_ENOMEM with the state of the
 * call's start (md_workspace_needed, md_set_workspace, then call again).  A
 * graph replay cannot heal: the bit stays for md_status; md_build_cells then
 * grows the list, and the graph must be captured again. */
int md_build_cells(kamd_ctx *ctx);

/* Forces at the current positions, Eq. (KAFix) with the truncation of
 * Eq. (VshiftedKALJ) (strict r < r_c(ab)).  The accelerations (m = 1) are
 * kept for the next step and exported to st->ax.. when auto_sync is on.
 * With KAMD_F_ENERGY and/or KAMD_F_VIRIAL, obs_dev (device, FP64 [n_rep][2])
 * receives per replica the shifted potential energy sum_{i<j} V_ij^cutoff and
 * the virial W = sum_{i<j} r_ij . F_ij; obs_dev may be NULL otherwise. */
int md_forces(kamd_ctx *ctx, uint32_t flags, double *obs_dev);

/* nsteps velocity-Verlet steps in the order of Sec. II.D / Sec. III.E:
 * r += v dt + a dt^2/2, wrap, v += a dt/2, a = F(r), v += a dt/2
 * (Eqs. (velVerletPos),(velVerletVel)).  Syncs once at the end (the list
 * check of md_build_cells). */
int md_step_nve(kamd_ctx *ctx, int32_t nsteps);

/* nsteps steps at constant N, V, T.
 * mode KAMD_NVT_STOCHASTIC: the NVE step, then every n_reassign steps (counted
 * from the context's step counter) all velocities are redrawn with the
 * Maxwell-Boltzmann flow chart of Sec. II.E.1 (Sec. III.G).
 * mode KAMD_NVT_NOSE_HOOVER: Eqs. (Noseupdate_ri)-(Noseupdate_xiapprox) and
 * (ridotKVLRoman) of Appendix B with X = 3N and bath mass Q = 3 N T tau^2;
 * the friction xi and ln s persist in the context.  tau > 0 is required for
 * this mode; n_reassign > 0 for the stochastic mode. */
int md_step_nvt(kamd_ctx *ctx, int32_t nsteps, int32_t mode, int32_t n_reassign, double tau);

/* Add one radial-distribution measurement (Sec. VI.A.1) of the current
 * configuration to hist_dev (device, uint64 [n_rep][3][n_bins], pair rows AA,
 * AB, BB; accumulated, the caller zeroes it): for every unique pair the
 * minimum-image distance r, bin = int(r / dr), counted when bin < n_bins;
 * AA and BB rows add 2 per pair, AB adds 1.  Requires n_bins*dr <= L/2 for
 * every replica and n_bins <= 5120 (else KAMD_EINVAL).  Normalisation to
 * g_ab(r) (Eqs. (gAA), (gAB)) is left to the caller.  Asynchronous, allocates
 * nothing (the cell grid is chosen on the device inside the workspace), and
 * may be recorded in a stream capture. */
int md_rdf(kamd_ctx *ctx, double dr, int32_t n_bins, uint64_t *hist_dev);

/* Mean-square displacement (Eqs. (msdwithi),(msdtw)) with unwrapped
 * coordinates (Sec. VI.B.1).  op 0 (SET_ORIGIN): store the current unwrapped
 * positions as origin `slot` (0 <= slot < msd_slots of the configuration, 16
 * by default; else KAMD_EINVAL).  op 1 (MEASURE): out_dev
 * (device, FP64 [n_rep][2]) receives per replica {msd_A, msd_B} against origin
 * `slot`. */
int md_msd(kamd_ctx *ctx, int32_t op, int32_t slot, double *out_dev);

/* Self part of the van Hove correlation function (the time generalisation
 * of g(r) named at the end of Sec. VI.A; definition of Hansen and McDonald):
 * adds to hist_dev (device, uint64 [n_rep][2][n_bins], A row then B row;
 * accumulated, the caller zeroes it) the count of particles whose unwrapped
 * displacement r = |r_u - r_u(origin slot)| has int(r / dr) = bin < n_bins.
 * The origin is set with md_msd(SET_ORIGIN).  KAMD_EINVAL for a slot outside
 * [0, msd_slots), dr < 1e-6 or n_bins outside [1, 1024].  Asynchronous. */
int md_van_hove(kamd_ctx *ctx, int32_t slot, double dr, int32_t n_bins, uint64_t *hist_dev);

/* Change the bath temperature of every replica (host, FP64 [n_rep], each
 * finite and > 0), as between the stages of a temperature ladder (Sec. V):
 * later stochastic-bath redraws and Nose-Hoover calls use it (a Nose-Hoover
 * call recomputes Q = 3 N T tau^2).  A captured Nose-Hoover graph keeps the Q
 * of its capture.  Syncs. */
int md_set_temperature(kamd_ctx *ctx, const double *temperature);

/* Multiply every velocity of replica r by factor[r] (host, FP64 [n_rep],
 * finite, >= 0), as for rescaling to a target total energy after a bath run
 * (Sec. V; Appendix exercises).  Forces are unchanged.  Syncs. */
int md_scale_velocities(kamd_ctx *ctx, const double *factor);

/* Log-spaced measurement steps for the MSD (Sec. VI.B.1, Eqs.
 * (logtimessteps), (A)): A = (n_md / t0)^(1/kmax), t_0 = t0, t_{k+1} = A t_k;
 * the steps are the distinct values round(t_k) (round half to even) in
 * [1, n_md], in increasing order.  Host only, no context.  Writes up to
 * max_out steps to out (host, may be NULL when max_out is 0) and the total
 * count to *count.  KAMD_EINVAL for n_md < 1, t0 < 0.5, kmax < 1. */
int md_log_schedule(int32_t n_md, double t0, int32_t kmax, int32_t *out, int32_t max_out, int32_t *count);

/* Sampled observables (the quantities the paper follows along a run: kinetic,
 * potential and total energy, Sec. III.F and Eq. (EsysNpart); temperature,
 * Eq. (equip3N)).  Rows written on the device every cfg.sample_every steps
 * (eager steps and graph replays alike).  host_out (host, FP64
 * [n_rep][max_rows][6]) receives, per replica, the most recent
 * rows = min(max_rows, rows held) samples in chronological order, each
 * {step, KE, PE, E_tot, T, W}: KE = sum v^2/2, PE the potential energy (shifted
 * unless pe_unshifted), E_tot = KE + PE, T = 2 KE / (d N), W the virial.
 * *rows receives the count (0 when sampling is off).  Syncs. */
int md_observables(kamd_ctx *ctx, double *host_out, int32_t max_rows, int32_t *rows);

/* Forget every sampled row (the next sample starts the ring again). */
int md_clear_samples(kamd_ctx *ctx);

/* Observables of the current state per replica into host_out (host, FP64
 * [n_rep][6]): {KE, PE, W, T, E_tot, P} with KE = sum v^2/2, PE the shifted
 * potential, T = 2 KE / (3N) (Eq. (equip3N)), E_tot = KE + PE (Eq.
 * (EsysNpart)) and pressure P = N T / V + W / (3V).  Runs one energy pass of
 * the force kernel.  Syncs. */
int md_observables_now(kamd_ctx *ctx, double *host_out);

/* Nose-Hoover state per replica into host_out (host, FP64 [n_rep][2]):
 * {xi, ln s}.  Syncs. */
int md_thermostat_state(kamd_ctx *ctx, double *host_out);

/* Write the internal state to the caller-order arrays given to md_init. */
int md_sync(kamd_ctx *ctx);

/* Re-read positions, velocities and image counters from the caller-order
 * arrays (after the caller changed them), recompute forces. */
int md_import(kamd_ctx *ctx);

/* Record nsteps steps of md_step_nve (ensemble 0) or md_step_nvt (ensemble 1,
 * with mode/n_reassign/tau) into a HIP graph held by the context, replacing
 * any earlier one.  Rebuild decisions stay on the device.  Nothing is
 * executed.  md_graph_launch(ctx) replays it on the context stream. */
int md_graph_capture(kamd_ctx *ctx, int32_t nsteps, int32_t ensemble, int32_t mode,
                     int32_t n_reassign, double tau);
int md_graph_launch(kamd_ctx *ctx);

/* Tuning of the list and of the step kernel, on a copy of the current state
 * that is restored afterwards.  A candidate is timed as the median of three
 * runs of probe_steps NVE steps, or of as many as take about 10 ms if that is
 * more (after a timed warm-up of probe_steps / 4).  Stage
 * 1 times each skin (0.2 .. min(0.5, L/2 - r_c,max)) with each cell division
 * (1, 2) on the current step kernel; stage 2 times, at the list parameters
 * kept, the step kernel with 256, 128 and 64 threads per block and, in the
 * mixed precisions, with windows off and on (md_set_force_kernel).  In each
 * stage the first candidate in that order within 1% of the stage's fastest is
 * kept (the smallest skin, the coarser grid, the direct kernel, the larger
 * block): ties are broken the same way on every run.  Candidates whose list
 * overflows are skipped.  Results in host_out (host, FP64 [5]): {skin,
 * cell_div, ms_per_step of the kept candidate, windows, threads per block};
 * the context keeps them.  KAMD_ENOMEM when a caller-owned workspace cannot
 * hold every candidate (md_workspace_needed then gives the size).  Syncs. */
int md_autotune(kamd_ctx *ctx, int32_t probe_steps, double *host_out);

/* Change skin and cell division (forces a rebuild at the next step).  With
 * cell_div 1 a replica may build its lists with a smaller skin, down to two
 * thirds of the given one, where that gives its box more cells per edge and
 * (cell-volume ratio) x (smaller skin / skin) is 1.15 or more: small boxes,
 * whose cells are otherwise well over a list radius wide.  The largest such
 * skin is taken, and the replica's rebuild test uses it too.  md_stats
 * reports the smallest skin in use.  The forces do not depend on the skin. */
int md_set_list_params(kamd_ctx *ctx, double skin, int32_t cell_div);

/* Step-kernel variant.  windows (mixed precisions): 1 gathers
 * the neighbours of a list part from LDS copies of the wavefront's stencil
 * rows, up to 4 groups of consecutive rows staged one after the other, when
 * they fit (the list then stores 16-bit offsets into them), 0 gathers every
 * neighbour from global memory (the default); a change forces a rebuild at
 * the next step.  wg_size: threads per block of the step kernel, 64, 128 or 256
 * (0 keeps the current one; 256 by default).  The forces are the same either
 * way (bit for bit with MIXED_FIXED).  Drops a captured graph.  KAMD_EINVAL
 * for windows = 1 in FP64.  Syncs. */
int md_set_force_kernel(kamd_ctx *ctx, int32_t windows, int32_t wg_size);

/* Statistics: host_out (host, FP64 [14]) = {steps, rebuilds, n_total,
 * list_rows, mean_list_len, max_list_len, skin, cell_div, mean_list_bytes,
 * windows (the force-kernel variant), fraction of list parts gathered from a
 * window, step-kernel threads per block, mean_walked, skin_min (the smallest
 * skin a replica uses; see md_set_list_params)}.  List lengths count
 * partners at the last build (without wavefront padding); mean_list_bytes is
 * their stored size per particle (4 bytes per 32-bit entry, 2 per 16-bit
 * entry); mean_walked is the number of entries the force kernels walk per
 * particle, each list part padded to its wavefront's longest.  Syncs. */
int md_stats(kamd_ctx *ctx, double *host_out);

/* Checkpoint: the full dynamical state (positions, velocities, forces, image
 * counters, thermostat variables, step counter) in caller order, as a host
 * blob.  With blob == NULL, *bytes receives the size.  Syncs. */
int md_get_state(kamd_ctx *ctx, void *blob, size_t *bytes);
int md_set_state(kamd_ctx *ctx, const void *blob, size_t bytes);

/* Measurement: nsteps NVE steps run eagerly on the context stream with HIP
 * events around every force-kernel launch and every streaming (drift/kick)
 * launch.  host_out (host, FP64 [8]) = {mean force-kernel ms, mean streaming
 * ms per step, total ms, list rebuilds during the run, ordered pairs inside
 * the cutoff per force launch (from a closing energy pass), steps, mean
 * rebuild-chain ms per step, 0}.  Syncs. */
int md_profile(kamd_ctx *ctx, int32_t nsteps, double *host_out);

/* Synchronise the stream and report the sticky device error word (KAMD_DEV_*
 * bits) in *word; returns KAMD_EDEVICE when it is non-zero.  Syncs. */
int md_status(kamd_ctx *ctx, uint32_t *word);

/* Clear the sticky device error word (after md_status reported it and the
 * caller dealt with the cause, e.g. relaxed a runaway start with a smaller
 * time step, Sec. II.F).  Syncs. */
int md_clear_status(kamd_ctx *ctx);

/* Message of the last error on this context (or of the last failed md_init
 * when ctx is NULL).  Never NULL. */
const char *md_last_error(const kamd_ctx *ctx);

/* Release the context and its device memory (waits for the stream). */
int md_destroy(kamd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* KAMD_H */
