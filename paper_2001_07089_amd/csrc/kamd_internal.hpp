// kamd_internal.hpp -- internal layout shared by the host runtime and the HIP
// kernels of the Kob-Andersen MD library (not part of the public ABI).
//
// Internal particle order ("slots").  Each replica r contributes two
// segments, its A particles then its B particles, each padded to a multiple of
// the 64-lane wavefront.  Every wavefront therefore covers particles of one
// replica and one type, so the box, the pair parameters of its rows and its
// reductions are wavefront-uniform (the type-split loops of the paper's
// acceleration routine, Sec. III.D, mapped onto waves).  Within a segment the
// particles are kept sorted by list cell (stable counting sort), which gives
// coalesced streaming and cache-local neighbour gathers.  Padding slots have
// id = -1, zero state, no list entries and are never anybody's neighbour.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kamd.h"

namespace kamd {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;               // threads per block for slot kernels
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;
constexpr int LIST_ROW_ALIGN = 4;        // neighbour rows are padded to this multiple
constexpr int CELL_SUBX = 4;             // list cells are sorted in sub-cells of a quarter
                                         // cell edge along x (cell_count/start/end per sub-cell)
constexpr int VH_MAX_BINS = 1024;       // bins of the self van Hove histogram
constexpr int SCAN_CHUNK = 2048;         // cells per block of the cell-range scan
constexpr int LIST_UNROLL = 8;           // candidates per step of the list builder's scan
// Force-kernel windows (mixed precisions): per wavefront and list part at
// most STAGE_PIECES row pieces (9 stencil rows, each a main run and a wrapped
// end) in at most STAGE_GROUPS groups of consecutive rows; one group at a time
// is staged in LDS, at most STAGE_SLOTS positions of 12 bytes of which the
// last 64 hold the lanes' own positions.  7.5 KB per wavefront leaves room
// for 20 wavefronts per CU (160 KB of LDS).
constexpr int STAGE_PIECES = 18;
constexpr int STAGE_GROUPS = 4;
constexpr int STAGE_SLOTS = 640;

// Neighbour-list layout.  The list of wavefront w is a block of rows * 64
// ints; entry k of lane l sits at (k / 4) * 256 + l * 4 + k % 4 inside it:
// each lane's entries come in 16-byte chunks of four, and chunk g of all 64
// lanes is 1 KB contiguous.  A lane therefore writes its list 16 contiguous
// bytes at a time, and a wavefront reads four rows with one coalesced int4
// load per lane.
__host__ __device__ inline size_t list_index(int w, int rows, int k, int lane)
{
    return (size_t)w * rows * 64 + (size_t)(k >> 2) * 256 + (size_t)lane * 4 + (k & 3);
}
constexpr double FIX_SCALE = 67108864.0; // 2^26 fixed-point units per force unit
constexpr double FIX_MAGIC = 6755399441055744.0;  // 1.5 * 2^52

struct SegInfo {
    int32_t rep;    // replica
    int32_t type;   // 0 = A, 1 = B
    int32_t slot0;  // first slot
    int32_t n;      // particles
    int32_t npad;   // slots (multiple of WAVE)
    int32_t cell0;  // first cell of this segment's list grid
    int32_t ncell;  // nc^3 (planar: nc^2)
    int32_t pad_;
};

struct RepInfo {
    double L, invL;
    double T;
    uint64_t seed;
    int64_t caller_off;    // first caller-order index
    int32_t n, na;
    int32_t seg[2];        // segment indices (A, B)
    int32_t wave0, wave1;  // waves [wave0, wave1) of both segments
    int32_t nc;            // list cells per box edge
    double skin;
    double disp_thr2;      // rebuild when max |dr|^2 exceeds this (real units)
    double run2;           // a single step's |dr|^2 beyond this is a runaway (real units)
    // pair constants in the u32 fixed-point length unit h = L / 2^32
    float rc2_fx[3];       // r_c(ab)^2 / h^2
    float rl2_fx[3];       // (r_c(ab) + skin)^2 / h^2, slightly enlarged
    float sig2_fx[3];      // sigma(ab)^2 / h^2
    float ir2_lim_fx[3];   // h^2 / r_lim(ab)^2: a pair closer than r_lim has a force whose
                           // 2^-26-unit rounding in MIXED_FIXED is no longer exact
    double c48_h[3];       // 48 eps(ab) / h: converts the fixed-unit sum to a force
    double fix_k[3];       // 48 eps(ab) / h * FIX_SCALE
    double fx_to_len;      // h
};

// Pair model in real units (binary64), AA/AB/BB.
struct Model {
    double eps[3];
    double sig2[3];
    double rc2[3];
    double vshift[3];
};

// Per-replica device-side mutable scalars.
struct RepDyn {
    double xi, lns, xia;  // Nose-Hoover friction, ln s, xi_approx for the running step
    double K2;            // sum v^2 at the start of the running step
    double c_kick;        // half-kick factor of the running step
    double pad[3];
};

// All device pointers, passed by value to kernels.
struct Dev {
    // slot-order state
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az;
    int32_t *img;         // [3][npad_total]
    int32_t *id;          // caller global index or -1
    uint4 *mirror;        // u32 fixed-point positions (x, y, z, 0)
    uint4 *mbuild;        // mirror at the last list build
    double4 *pos4;        // FP64 only (else null): positions (x, y, z, 0) packed for the force kernel's gathers
    // permutation scratch (same layout)
    double *sx, *sy, *sz, *svx, *svy, *svz, *sax, *say, *saz;
    int32_t *simg, *sid;
    uint4 *smirror;
    // layout tables
    const SegInfo *seg;
    const RepInfo *rep;
    const int32_t *wave_seg;
    // cells and lists
    int32_t *cell_of, *rank, *cell_count, *cell_start, *cell_end, *order;
    int32_t *rb_force;    // per replica: rebuild at the next check regardless
    int32_t *rb_any;      // [2]: [0] the number of waves that rebuild this step (gate kernel)
    int32_t *rb_wlist;    // [nwaves]: those waves, replica by replica (gate kernel)
    uint32_t *maxdisp;    // per replica: max |r - r_build|^2 (float bits) since the last check
    int32_t *nbr;         // per wave: rows x 64 entries, see list_index
    int2 *kmax;           // per wave: entries of the A part, entries of the B part
    int2 *lbase;          // per wave and part: base slot of 16-bit entries, -1 for 32-bit entries,
                          // or -2 - W: 16-bit offsets into a staged window of W slots
    int2 *pieces;         // per wave and part: STAGE_PIECES (first slot, slots) of the window's pieces
    int4 *sgroups;        // per wave and part: STAGE_GROUPS (end of its pieces, window slots, end of its entries, -)
    int2 *pcount;         // per wave: window groups of the A part and of the B part (0: not staged)
    int32_t stage_ok;     // the force kernels stage windows (mixed precisions)
    int32_t *nlen;        // per slot: true list length (stats)
    // reductions
    double *wred;         // per wave [4]
    double *rsum;         // per replica [4]
    double *obs;          // per replica [8]: KE2, PE, W, -, ...
    RepDyn *dyn;
    uint32_t *err;
    int32_t *counters;    // [0] = rebuilds, [1] = device step counter
    // RDF scratch; rdf_grid[r] = {cells per edge, first cell, cells} of the
    // last measurement's grid; rdf_count / rdf_start hold rdf_cells_cap cells
    int32_t *rdf_cell_of, *rdf_rank, *rdf_count, *rdf_start;
    double4 *rdf_pos;
    int4 *rdf_grid;
    int64_t rdf_cells_cap;
    const int32_t *rdf_block_rep;
    const int32_t *rdf_block_start;
    // MSD origins [msd_slots][3][n_total] in caller order
    double *origin;
    int32_t msd_slots;
    // sampled observables [nrep][ring_cap][6]: step, KE, PE, E_tot, T, W
    // (null when sampling is off); counters[2] counts the rows written
    double *ring;
    int32_t ring_cap;
    // sizes
    int32_t npad_total;
    int32_t n_total;
    int32_t nwaves;
    int32_t nrep;
    int32_t dim;          // 3, or 2 for a planar system (z = vz = 0)
    int32_t ncells;
    int32_t rows;         // neighbour-list row capacity
    int32_t scan_cps;     // scan chunks (SCAN_CHUNK cells) of the largest segment
    int32_t *chunk_sum;   // [nseg][scan_cps]: particles of each scan chunk (segments of several chunks)
};


// The static workspace (static_ws.hip): the runtime tells it when a context
// that used a device's array is destroyed.
void release_static_workspace(int device);
void set_init_error(const char *msg);
void mark_static(kamd_ctx *c, int device);

// ---------------------------------------------------------------- launchers
// Each returns hipGetLastError() after its launch(es).
hipError_t launch_rb_gate(const Dev &d, hipStream_t s);
hipError_t launch_rb_assign(const Dev &d, hipStream_t s);
hipError_t launch_rb_scan(const Dev &d, int nseg, hipStream_t s);
hipError_t launch_rb_scatter(const Dev &d, hipStream_t s);
hipError_t launch_rb_sortgather(const Dev &d, hipStream_t s);
hipError_t launch_rb_list(const Dev &d, int cell_div, hipStream_t s);

// The force kernel also closes the step's rebuild check (resets maxdisp and
// rb_force) and, with step_inc, advances the device step counter.
hipError_t launch_force(const Dev &d, const Model &m, int prec, bool energy, bool step_inc, hipStream_t s);
// NVE: forces fused with the closing half kick and the next drift (new
// mirror into mirror_out, displacement maximum into md_out; FP64 also the
// packed positions into pos4_out, which must differ from d.pos4 and is
// ignored by the mixed precisions).
// With energy, also the per-wave partials wred[0..3] = {sum v(t)^2, PE, W,
// pairs} of the step's end state (v(t) is the closed half kick).
// wpb: wavefronts per block of the step kernel (1, 2 or 4; an autotuner axis).
hipError_t launch_force_kd(const Dev &d, const Model &m, int prec, double dt, uint4 *mirror_out, uint32_t *md_out,
                           double4 *pos4_out, bool energy, int wpb, hipStream_t s);
// Pack d.x, d.y, d.z into d.pos4 (every slot, padding included).
hipError_t launch_pack_pos(const Dev &d, hipStream_t s);

hipError_t launch_drift(const Dev &d, double dt, hipStream_t s);
hipError_t launch_drift_nh(const Dev &d, double dt, hipStream_t s);
hipError_t launch_kick_nve(const Dev &d, double dt, bool want_ke, hipStream_t s);
hipError_t launch_kick_nh(const Dev &d, hipStream_t s);
hipError_t launch_kick_drift(const Dev &d, double dt, bool want_ke, hipStream_t s);
hipError_t launch_rep_reduce(const Dev &d, int mask, hipStream_t s);
hipError_t launch_nh_begin(const Dev &d, double dt, const double *Q, hipStream_t s);
hipError_t launch_nh_end(const Dev &d, double dt, const double *Q, hipStream_t s);
hipError_t launch_set_k2(const Dev &d, hipStream_t s);
hipError_t launch_mb_draw(const Dev &d, uint32_t tag, hipStream_t s);
hipError_t launch_mb_draw_dev(const Dev &d, hipStream_t s);
hipError_t launch_mb_center(const Dev &d, hipStream_t s);
hipError_t launch_mb_scale(const Dev &d, hipStream_t s);
hipError_t launch_scale_v(const Dev &d, const double *f, hipStream_t s);
hipError_t launch_ke_partial(const Dev &d, hipStream_t s);

hipError_t launch_import(const Dev &d, const double *const *arr, const int32_t *img, hipStream_t s);
hipError_t launch_export(const Dev &d, double *const *arr, int32_t *img, hipStream_t s);
hipError_t launch_mirror(const Dev &d, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_store_obs(const Dev &d, double *out, hipStream_t s);
hipError_t launch_store_pe_w(const Dev &d, double *out, hipStream_t s);
// One row of the observables ring from rsum: mask 1 KE, 2 PE and W, 4 step,
// E_tot and T, then advance the row counter (counters[2]).
hipError_t launch_sample(const Dev &d, int mask, hipStream_t s);

// Grid set-up on the device (k_rdf_setup), counting sort by RDF cell.
hipError_t launch_rdf_prepare(const Dev &d, double rmax, hipStream_t s);
hipError_t launch_rdf(const Dev &d, double dr, int nbins, int nblocks, uint64_t *hist, hipStream_t s);
hipError_t launch_msd_set(const Dev &d, int slot, hipStream_t s);
hipError_t launch_msd_measure(const Dev &d, int slot, hipStream_t s);
hipError_t launch_msd_finish(const Dev &d, double *out, hipStream_t s);
hipError_t launch_van_hove(const Dev &d, int slot, double dr, int nbins, uint64_t *hist, hipStream_t s);

}  // namespace kamd
