// runtime.cpp -- host runtime of the Kob-Andersen MD library: the C ABI of
// include/kamd.h, the replica/slot/cell layout, device memory, the step
// loops, HIP graph capture, the list autotuner and checkpoints.
#include "kamd.h"
#include "kamd_internal.hpp"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

using namespace kamd;

static std::string g_init_error = "no error";

// Layout of the replicas in slot order and the list grid for one choice of
// skin and cell division.
struct Plan {
    std::vector<SegInfo> segs;
    std::vector<RepInfo> rinfo;
    std::vector<int32_t> wave_seg;
    int32_t npad = 0, nwaves = 0, ncells = 0, rows = 0, n_total = 0;
    int32_t scan_cps = 1;     // scan chunks of the largest segment
    int64_t ncells_wide = 0;  // the same count without 32-bit truncation
    bool fp64 = false;        // FP64 precision: two packed position buffers
};

// Sizes of the fixed part of a workspace (independent of the list parameters).
struct Shape {
    size_t np = 0, nt = 0, nwaves = 0, nrep = 0, nseg = 0;
    size_t rdf_blocks = 0;  // blocks of the RDF histogram kernel (BLOCK particles of one replica each)
    size_t rdf_cells = 0;   // RDF cell capacity: 2 n + 64 per replica
    size_t ring = 0;        // rows of the observables ring, all replicas
    size_t msd_slots = 16;
    bool fp64 = false;
};

struct kamd_ctx {
    kamd_config cfg{};
    Model model{};
    double rc_max = 0.0;
    std::vector<kamd_replica> reps;
    std::vector<SegInfo> segs;
    std::vector<RepInfo> rinfo;
    std::vector<int32_t> wave_seg;
    std::vector<int32_t> rdf_block_rep, rdf_block_start;
    kamd_state st{};
    hipStream_t stream = nullptr;
    int device = 0;
    Dev d{};
    // The device workspace: one block, the caller's (borrowed) or the
    // library's own when md_init was given none.  Layout: the fixed part
    // (everything whose size does not depend on the list parameters), then
    // the cell arrays and the neighbour list from list_off on.
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    size_t list_off = 0;              // end of the fixed part
    size_t need_bytes = 0;            // workspace the last refused request needed
    int32_t rows_floor = 0;           // list rows a healed overflow asked for
    uint4 *mirror_alt = nullptr;      // second u32 mirror (fused force+drift steps)
    double4 *pos4_alt = nullptr;      // second packed FP64 position buffer (FP64 fused steps)
    uint32_t *md_base = nullptr;      // [2][n_rep] displacement maxima
    double *Q_dev = nullptr;
    double *rep_arg = nullptr;        // per-replica host arguments staged for a kernel
    double *obs_stage = nullptr;      // device [n_rep][4]
    double *state_tmp = nullptr;      // device caller-order staging: checkpoints, list-heal snapshots
    int32_t *img_tmp = nullptr;
    RepDyn *dyn_snap = nullptr;       // thermostat scalars of a list-heal snapshot
    int32_t *cnt_snap = nullptr;      // device counters of a list-heal snapshot
    int64_t step = 0;
    int64_t rebuilds_host = 0;
    double skin = 0.3;
    int cell_div = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_steps = 0;
    Plan plan;                        // the current list parameters' layout
    Shape shape;                      // sizes of the workspace's fixed part
    int static_device = -1;           // >= 0: the workspace is that device's static array
    bool stage_windows = false;       // mixed-precision force kernels gather from LDS windows
    int force_wpb = WAVES_PER_BLOCK;  // wavefronts per block of the step kernel
    std::string err = "no error";
};

// ------------------------------------------------------------------ errors
static int fail(kamd_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_init_error = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), KAMD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ layout
static void model_from(const kamd_model &m, Model &out, double &rc_max)
{
    rc_max = 0.0;
    for (int p = 0; p < 3; ++p) {
        const double s = m.sigma[p];
        const double rc = m.rc_factor * s;
        out.eps[p] = m.eps[p];
        out.sig2[p] = s * s;
        out.rc2[p] = rc * rc;
        const double sr2 = (s * s) / (rc * rc);
        const double sr6 = sr2 * sr2 * sr2;
        out.vshift[p] = 4.0 * m.eps[p] * (sr6 * sr6 - sr6);
        rc_max = std::max(rc_max, rc);
    }
}

// Smallest separation at which the pair force of one pair type can still be
// rounded exactly to 2^-26 force units by the MIXED_FIXED kernels: the
// rounding adds the scaled component to 1.5 * 2^52, which is exact while
// |F| 2^26 < 2^51, i.e. |F| < 2^25.  The pair force magnitude
// 48 |eps| s6 |s6 - 1/2| / r (s6 = (sigma/r)^6, Eq. (KAFix)) falls
// monotonically on (0, 2^(1/6) sigma), so bisection finds where it crosses
// 2^25 (less a 2^-8 margin for the FP32 pair arithmetic).  0 when the model
// has no such crossing (eps = 0).
static double fixed_range_rmin(double eps, double sigma)
{
    const double flim = std::ldexp(1.0, 25) * (1.0 - std::ldexp(1.0, -8));
    auto F = [&](double r) {
        const double sr2 = (sigma / r) * (sigma / r);
        const double s6 = sr2 * sr2 * sr2;
        return 48.0 * std::fabs(eps) * s6 * std::fabs(s6 - 0.5) / r;
    };
    double lo = 1e-6 * sigma, hi = std::pow(2.0, 1.0 / 6.0) * sigma;
    if (!(F(lo) > flim)) return 0.0;
    for (int k = 0; k < 200; ++k) {
        const double mid = 0.5 * (lo + hi);
        if (F(mid) > flim) lo = mid;
        else hi = mid;
    }
    return hi;
}

static inline int dim_of(const kamd_config *cfg) { return cfg->dim == 2 ? 2 : 3; }

static int validate(kamd_ctx *c, const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep)
{
    if (!cfg || !reps || n_rep <= 0) return fail(c, KAMD_EINVAL, "null config/replicas or n_rep <= 0");
    if (cfg->precision < 0 || cfg->precision > 2) return fail(c, KAMD_EINVAL, "bad precision %d", cfg->precision);
    if (!(cfg->dt > 0.0)) return fail(c, KAMD_EINVAL, "dt must be > 0");
    if (cfg->cell_div < 0 || cfg->cell_div > 2) return fail(c, KAMD_EINVAL, "cell_div must be 0, 1 or 2");
    if (cfg->dim != 0 && cfg->dim != 2 && cfg->dim != 3) return fail(c, KAMD_EINVAL, "dim must be 0, 2 or 3");
    if (cfg->pe_unshifted != 0 && cfg->pe_unshifted != 1) return fail(c, KAMD_EINVAL, "pe_unshifted must be 0 or 1");
    if (cfg->sample_every < 0 || cfg->sample_capacity < 0 || cfg->sample_capacity > (1 << 24))
        return fail(c, KAMD_EINVAL, "sample_every must be >= 0 and sample_capacity in [0, 2^24]");
    if (cfg->msd_slots < 0 || cfg->msd_slots > 64) return fail(c, KAMD_EINVAL, "msd_slots must be in [0, 64]");
    if (!(cfg->model.rc_factor > 0.0)) return fail(c, KAMD_EINVAL, "rc_factor must be > 0");
    for (int p = 0; p < 3; ++p)
        if (!(cfg->model.sigma[p] > 0.0) || !std::isfinite(cfg->model.eps[p]))
            return fail(c, KAMD_EINVAL, "bad model parameters for pair %d", p);
    Model m;
    double rcmax;
    model_from(cfg->model, m, rcmax);
    int64_t expect_off = 0;
    for (int r = 0; r < n_rep; ++r) {
        const kamd_replica &R = reps[r];
        if (R.n <= 0 || R.n_a < 0 || R.n_a > R.n) return fail(c, KAMD_EINVAL, "replica %d: bad n=%d n_a=%d", r, R.n, R.n_a);
        if (R.offset != expect_off) return fail(c, KAMD_EINVAL, "replica %d: offset %lld, expected %lld (contiguous)", r, (long long)R.offset, (long long)expect_off);
        if (!(R.box > 0.0) || !std::isfinite(R.box)) return fail(c, KAMD_EINVAL, "replica %d: bad box", r);
        if (!(R.temperature >= 0.0)) return fail(c, KAMD_EINVAL, "replica %d: bad temperature", r);
        if (!(rcmax < 0.5 * R.box)) return fail(c, KAMD_EBOX, "replica %d: largest cutoff %.6g >= L/2 = %.6g", r, rcmax, 0.5 * R.box);
        expect_off += R.n;
    }
    if (expect_off > (int64_t)1 << 30) return fail(c, KAMD_EINVAL, "too many particles");
    return KAMD_OK;
}


// Limits of the list cell grid.  A segment holds at most 2^24 cells (nc is
// lowered to fit: wider cells stay correct, they only add candidates), and a
// plan at most 2^26 cells in all (52 bytes each with the sub-cell counters
// and ranges), which keeps every sub-cell index, scan offset and launch size
// far inside 32 bits.
constexpr int64_t MAX_SEG_CELLS = (int64_t)1 << 24;
constexpr int64_t MAX_PLAN_CELLS = (int64_t)1 << 26;

static int cell_cap(int dim) { return dim == 2 ? 4096 : 256; }  // nc^(dim) <= MAX_SEG_CELLS
// Skin per replica.  With one cell per list radius a box of edge L has
// floor(L / list radius) cells per edge, so in small boxes a cell can be up
// to twice the list radius wide, and every particle tests the particles of 9
// stencil rows of such cells.  A replica takes a smaller skin, no less than
// SKIN_TRIM times the requested one, where that buys more cells per edge and
// the list build's work per step falls by CELL_GAIN or more: the candidates
// per build fall as the cell volume, the builds grow as 1 / skin (the largest
// skin that gets the extra cells is taken).  The pair set within the
// cutoff, and so every force, does not depend on it.
constexpr double SKIN_TRIM = 2.0 / 3.0;
constexpr double CELL_GAIN = 1.15;

static double list_skin(const kamd_config *cfg) { return cfg->skin < 0.0 ? 0.3 : cfg->skin; }

// Rows per replica of the observables ring (0 when sampling is off).
static int ring_rows(const kamd_config *cfg)
{
    if (cfg->sample_every <= 0) return 0;
    return cfg->sample_capacity > 0 ? cfg->sample_capacity : 1024;
}

static void make_plan(const kamd_config *cfg, const kamd_replica *reps, int n_rep, double skin, int cell_div,
                      Plan &P, int rows_floor = 0)
{
    Model m;
    double rcmax;
    model_from(cfg->model, m, rcmax);
    const int reach = cell_div <= 0 ? 1 : cell_div;
    const double cap = cfg->list_capacity > 0.0 ? cfg->list_capacity : 1.6;
    P = Plan();
    P.fp64 = cfg->precision == KAMD_PREC_FP64;
    const bool planar = dim_of(cfg) == 2;
    auto cells_per_edge = [&](double box, double s) {
        return (int)std::max(1.0, std::min(std::floor(box * reach / (rcmax + s)), (double)cell_cap(dim_of(cfg))));
    };
    auto rep_skin = [&](double box) {
        if (reach != 1 || !(skin > 0.0)) return skin;
        const double lo = SKIN_TRIM * skin;
        const int n0 = cells_per_edge(box, skin), n1 = cells_per_edge(box, lo);
        if (n1 < 3 || n1 <= n0) return skin;
        double s = std::min(skin, box / n1 - rcmax);  // the largest skin with n1 cells, up to rounding
        while (s > lo && cells_per_edge(box, s) < n1) s = std::nextafter(s, 0.0);
        s = std::max(s, lo);
        return std::pow((double)n1 / n0, planar ? 2 : 3) * (s / skin) >= CELL_GAIN ? s : skin;
    };
    std::vector<double> rskin(n_rep);
    for (int r = 0; r < n_rep; ++r) {  // the grid size first (an oversize plan is refused)
        rskin[r] = rep_skin(reps[r].box);
        const int64_t nc = cells_per_edge(reps[r].box, rskin[r]);
        P.ncells_wide += 2 * (planar ? nc * nc : nc * nc * nc);
    }
    const bool fits = P.ncells_wide <= MAX_PLAN_CELLS;
    int32_t slot = 0, cell = 0;
    double rows_need = 0.0;
    for (int r = 0; r < n_rep; ++r) {
        const kamd_replica &K = reps[r];
        RepInfo R;
        std::memset(&R, 0, sizeof R);
        R.L = K.box;
        R.invL = 1.0 / K.box;
        R.T = K.temperature;
        R.seed = K.seed;
        R.caller_off = K.offset;
        R.n = K.n;
        R.na = K.n_a;
        const double skin_r = rskin[r];
        R.skin = skin_r;
        const double half = 0.5 * skin_r;
        R.disp_thr2 = half * half * (1.0 - 1e-5);
        // a move of half the smallest sigma in one step (a normal step moves
        // about a hundredth of that) marks an unstable, runaway integration
        const double smin = std::min(cfg->model.sigma[0], std::min(cfg->model.sigma[1], cfg->model.sigma[2]));
        R.run2 = 0.25 * smin * smin;
        const int nc = cells_per_edge(K.box, skin_r);
        R.nc = nc;
        const double h = K.box / 4294967296.0;
        for (int p = 0; p < 3; ++p) {
            const double rc = cfg->model.rc_factor * cfg->model.sigma[p];
            const double rl = rc + skin_r;
            R.rc2_fx[p] = (float)((rc / h) * (rc / h));
            R.rl2_fx[p] = (float)((rl / h) * (rl / h) * (1.0 + 4e-6));
            R.sig2_fx[p] = (float)((cfg->model.sigma[p] / h) * (cfg->model.sigma[p] / h));
            R.c48_h[p] = 48.0 * cfg->model.eps[p] / h;
            R.fix_k[p] = R.c48_h[p] * FIX_SCALE;
            // a pair is flagged when its 1/r^2 (fixed units) exceeds this; the
            // 1e-5 margin covers the rounding of the device's FP32 reciprocal
            const double rmin = fixed_range_rmin(cfg->model.eps[p], cfg->model.sigma[p]);
            R.ir2_lim_fx[p] = rmin > 0.0 ? (float)((h / rmin) * (h / rmin) * (1.0 - 1e-5)) : INFINITY;
        }
        R.fx_to_len = h;
        R.wave0 = slot / WAVE;
        for (int t = 0; t < 2; ++t) {
            SegInfo S;
            std::memset(&S, 0, sizeof S);
            S.rep = r;
            S.type = t;
            S.slot0 = slot;
            S.n = t == 0 ? K.n_a : K.n - K.n_a;
            S.npad = (S.n + WAVE - 1) / WAVE * WAVE;
            S.cell0 = cell;
            // a planar system keeps every particle at z = 0: one layer of cells
            S.ncell = planar ? nc * nc : nc * nc * nc;
            R.seg[t] = (int32_t)P.segs.size();
            for (int w = 0; w < S.npad / WAVE; ++w) P.wave_seg.push_back(R.seg[t]);
            slot += S.npad;
            cell += fits ? S.ncell : 0;
            P.scan_cps = std::max(P.scan_cps, (S.ncell + SCAN_CHUNK - 1) / SCAN_CHUNK);
            P.segs.push_back(S);
        }
        R.wave1 = slot / WAVE;
        P.rinfo.push_back(R);
        // expected list rows: wavefront maxima of the A part and the B part
        // (planar: number density per area, disc area)
        const double V = planar ? K.box * K.box : K.box * K.box * K.box;
        const double rhoA = K.n_a / V, rhoB = (K.n - K.n_a) / V;
        const double pi43 = 4.0 / 3.0 * M_PI;
        auto vol = [&](int p) {
            double rl = cfg->model.rc_factor * cfg->model.sigma[p] + skin_r;
            return planar ? M_PI * rl * rl : pi43 * rl * rl * rl;
        };
        const double rowsA = std::max(K.n_a > 0 ? rhoA * vol(0) + rhoB * vol(1) : 0.0,
                                      K.n > K.n_a ? rhoA * vol(1) + rhoB * vol(2) : 0.0);
        rows_need = std::max(rows_need, rowsA);
        P.n_total += K.n;
    }
    P.npad = slot;
    P.nwaves = slot / WAVE;
    P.ncells = cell;
    int rows = std::max((int)std::ceil(cap * rows_need) + 32, rows_floor);
    rows = (rows + LIST_ROW_ALIGN - 1) / LIST_ROW_ALIGN * LIST_ROW_ALIGN;
    P.rows = rows;
}

static int plan_fits(kamd_ctx *c, const Plan &P)
{
    if (P.ncells_wide > MAX_PLAN_CELLS)
        return fail(c, KAMD_EINVAL, "list cell grid of %lld cells exceeds the limit of %lld (fewer or smaller replicas)",
                    (long long)P.ncells_wide, (long long)MAX_PLAN_CELLS);
    return KAMD_OK;
}

// ------------------------------------------------------------------ memory
// Bump allocator over the device workspace (256-byte aligned pieces).  With no
// base it only measures: md_workspace_size and md_admit run the very carve
// that md_init performs, so the sizes they report are the sizes used.
struct Carve {
    char *base = nullptr;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

static int msd_slots_of(const kamd_config *cfg) { return cfg->msd_slots > 0 ? cfg->msd_slots : 16; }

static Shape shape_of(const kamd_config *cfg, const kamd_replica *reps, int n_rep, const Plan &P)
{
    Shape z;
    z.np = P.npad;
    z.nt = P.n_total;
    z.nwaves = P.nwaves;
    z.nrep = n_rep;
    z.nseg = P.segs.size();
    for (int r = 0; r < n_rep; ++r) {
        z.rdf_blocks += (reps[r].n + BLOCK - 1) / BLOCK;
        z.rdf_cells += 2 * (size_t)reps[r].n + 64;
    }
    z.ring = (size_t)ring_rows(cfg) * n_rep;
    z.msd_slots = msd_slots_of(cfg);
    z.fp64 = cfg->precision == KAMD_PREC_FP64;
    return z;
}

// Pieces of the fixed part that the context holds outside Dev.
struct CtxBufs {
    uint4 *mirror_alt = nullptr;
    double4 *pos4_alt = nullptr;
    uint32_t *md_base = nullptr;
    double *Q_dev = nullptr, *rep_arg = nullptr, *obs_stage = nullptr, *state_tmp = nullptr;
    int32_t *img_tmp = nullptr;
    RepDyn *dyn_snap = nullptr;
    int32_t *cnt_snap = nullptr;
    int32_t *rdf_block_rep = nullptr, *rdf_block_start = nullptr;
};

// The fixed part: slot-order state and its permutation scratch, layout
// tables, rebuild bookkeeping, reductions, observables ring, MSD origins, RDF
// scratch, caller-order staging.
static void carve_fixed(Dev &d, CtxBufs &b, const Shape &z, Carve &k)
{
    const size_t np = z.np, nt = z.nt;
    double **f64[] = {&d.x, &d.y, &d.z, &d.vx, &d.vy, &d.vz, &d.ax, &d.ay, &d.az,
                      &d.sx, &d.sy, &d.sz, &d.svx, &d.svy, &d.svz, &d.sax, &d.say, &d.saz};
    for (auto p : f64) *p = k.take<double>(np);
    d.img = k.take<int32_t>(3 * np);
    d.simg = k.take<int32_t>(3 * np);
    d.id = k.take<int32_t>(np);
    d.sid = k.take<int32_t>(np);
    d.mirror = k.take<uint4>(np);
    d.mbuild = k.take<uint4>(np);
    d.smirror = k.take<uint4>(np + LIST_UNROLL);  // the list scan reads up to 7 past a range
    b.mirror_alt = k.take<uint4>(np);
    d.pos4 = z.fp64 ? k.take<double4>(np) : nullptr;
    b.pos4_alt = z.fp64 ? k.take<double4>(np) : nullptr;
    d.seg = k.take<SegInfo>(z.nseg);
    d.rep = k.take<RepInfo>(z.nrep);
    d.wave_seg = k.take<int32_t>(z.nwaves);
    d.cell_of = k.take<int32_t>(np);
    d.rank = k.take<int32_t>(np);
    d.order = k.take<int32_t>(np);
    d.nlen = k.take<int32_t>(np);
    d.rb_force = k.take<int32_t>(z.nrep);
    d.rb_any = k.take<int32_t>(2);
    d.rb_wlist = k.take<int32_t>(z.nwaves);
    b.md_base = k.take<uint32_t>(2 * z.nrep);
    d.kmax = k.take<int2>(z.nwaves);
    d.lbase = k.take<int2>(z.nwaves);
    d.pieces = k.take<int2>(z.nwaves * 2 * STAGE_PIECES);
    d.sgroups = k.take<int4>(z.nwaves * 2 * STAGE_GROUPS);
    d.pcount = k.take<int2>(z.nwaves);
    d.wred = k.take<double>(4 * z.nwaves);
    d.rsum = k.take<double>(4 * z.nrep);
    d.obs = k.take<double>(8 * z.nrep);
    d.dyn = k.take<RepDyn>(z.nrep);
    d.err = k.take<uint32_t>(4);
    d.counters = k.take<int32_t>(8);
    b.Q_dev = k.take<double>(z.nrep);
    b.rep_arg = k.take<double>(z.nrep);
    b.obs_stage = k.take<double>(4 * z.nrep);
    d.ring = z.ring ? k.take<double>(6 * z.ring) : nullptr;
    d.origin = k.take<double>(z.msd_slots * 3 * nt);
    d.rdf_cell_of = k.take<int32_t>(np);
    d.rdf_rank = k.take<int32_t>(np);
    d.rdf_pos = k.take<double4>(nt);
    d.rdf_count = k.take<int32_t>(z.rdf_cells);
    d.rdf_start = k.take<int32_t>(z.rdf_cells);
    d.rdf_grid = k.take<int4>(z.nrep);
    b.rdf_block_rep = k.take<int32_t>(z.rdf_blocks);
    b.rdf_block_start = k.take<int32_t>(z.rdf_blocks);
    b.state_tmp = k.take<double>(9 * nt);
    b.img_tmp = k.take<int32_t>(3 * nt);
    b.dyn_snap = k.take<RepDyn>(z.nrep);
    b.cnt_snap = k.take<int32_t>(8);
}

// The part that depends on the list parameters: per sub-cell counters and
// ranges, the scan chunk totals and the neighbour list.
static void carve_list(Dev &d, const Plan &P, Carve &k)
{
    const size_t nsub = (size_t)CELL_SUBX * P.ncells;
    d.cell_count = k.take<int32_t>(nsub);
    d.cell_start = k.take<int32_t>(nsub);
    d.cell_end = k.take<int32_t>(nsub);
    d.chunk_sum = k.take<int32_t>(P.segs.size() * (size_t)P.scan_cps);
    d.nbr = k.take<int32_t>((size_t)P.rows * P.npad);
}

static size_t fixed_bytes(const Shape &z)
{
    Dev d{};
    CtxBufs b;
    Carve k;
    carve_fixed(d, b, z, k);
    return (k.off + 255) & ~(size_t)255;
}

static size_t list_bytes(const Plan &P)
{
    Dev d{};
    Carve k;
    carve_list(d, P, k);
    return k.off;
}

extern "C" int md_workspace_size(const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep, size_t *bytes)
{
    int rc = validate(nullptr, cfg, reps, n_rep);
    if (rc) return rc;
    if (!bytes) return fail(nullptr, KAMD_EINVAL, "bytes is null");
    Plan P;
    make_plan(cfg, reps, n_rep, list_skin(cfg), cfg->cell_div <= 0 ? 1 : cfg->cell_div, P);
    rc = plan_fits(nullptr, P);
    if (rc) return rc;
    *bytes = fixed_bytes(shape_of(cfg, reps, n_rep, P)) + list_bytes(P);
    return KAMD_OK;
}

extern "C" int md_admit(const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep, size_t budget,
                        int32_t *admitted, int32_t *n_admitted)
{
    if (!cfg || !reps || n_rep <= 0 || !admitted) return fail(nullptr, KAMD_EINVAL, "bad arguments to md_admit");
    int cnt = 0;
    std::vector<kamd_replica> acc;
    int64_t off = 0;
    for (int r = 0; r < n_rep; ++r) {
        kamd_replica k = reps[r];
        k.offset = off;
        acc.push_back(k);
        size_t b = 0;
        int v = validate(nullptr, cfg, acc.data(), (int)acc.size());
        if (v == KAMD_OK) {
            Plan P;
            make_plan(cfg, acc.data(), (int)acc.size(), list_skin(cfg), cfg->cell_div <= 0 ? 1 : cfg->cell_div, P);
            if (P.ncells_wide > MAX_PLAN_CELLS) v = KAMD_EINVAL;
            else b = fixed_bytes(shape_of(cfg, acc.data(), (int)acc.size(), P)) + list_bytes(P);
        }
        if (v == KAMD_OK && b <= budget) {
            admitted[r] = 1;
            off += k.n;
            ++cnt;
        } else {
            admitted[r] = 0;
            acc.pop_back();
        }
    }
    if (n_admitted) *n_admitted = cnt;
    return KAMD_OK;
}

#define TRY(x)                 \
    do {                       \
        int r_ = (x);          \
        if (r_) return r_;     \
    } while (0)

// Point Dev and the context's buffers into the workspace: the fixed part at
// its start, the cell arrays and the list of plan P from list_off on.
static void bind_workspace(kamd_ctx *c, const Plan &P)
{
    Dev &d = c->d;
    CtxBufs b;
    Carve k;
    k.base = c->ws;
    carve_fixed(d, b, c->shape, k);
    c->list_off = (k.off + 255) & ~(size_t)255;
    c->mirror_alt = b.mirror_alt;
    c->pos4_alt = b.pos4_alt;
    c->md_base = b.md_base;
    d.maxdisp = b.md_base;
    c->Q_dev = b.Q_dev;
    c->rep_arg = b.rep_arg;
    c->obs_stage = b.obs_stage;
    c->state_tmp = b.state_tmp;
    c->img_tmp = b.img_tmp;
    c->dyn_snap = b.dyn_snap;
    c->cnt_snap = b.cnt_snap;
    d.rdf_block_rep = b.rdf_block_rep;
    d.rdf_block_start = b.rdf_block_start;
    Carve kl;
    kl.base = c->ws + c->list_off;
    carve_list(d, P, kl);
    d.npad_total = P.npad;
    d.n_total = P.n_total;
    d.nwaves = P.nwaves;
    d.nrep = (int32_t)c->reps.size();
    d.dim = dim_of(&c->cfg);
    d.rows = P.rows;
    d.ncells = P.ncells;
    d.scan_cps = P.scan_cps;
    d.rdf_cells_cap = (int64_t)c->shape.rdf_cells;
    d.stage_ok = c->cfg.precision != KAMD_PREC_FP64 && c->stage_windows;
    d.ring_cap = ring_rows(&c->cfg);
    d.msd_slots = (int32_t)c->shape.msd_slots;
}

static size_t need_for(const kamd_ctx *c, const Plan &P) { return c->list_off + list_bytes(P); }

// Zero what the kernels read before they write it (the fixed part).
static int init_fixed(kamd_ctx *c)
{
    Dev &d = c->d;
    const int64_t np = d.npad_total, nr = d.nrep, nw = d.nwaves;
    double *f64[] = {d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az,
                     d.sx, d.sy, d.sz, d.svx, d.svy, d.svz, d.sax, d.say, d.saz};
    for (auto p : f64) HIPCHK(c, launch_zero_f64(p, np, c->stream));
    HIPCHK(c, launch_zero_i32(d.img, 3 * np, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.mirror, 4 * np, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.mbuild, 4 * np, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.smirror, 4 * (np + LIST_UNROLL), c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)c->mirror_alt, 4 * np, c->stream));
    HIPCHK(c, launch_zero_i32(d.nlen, np, c->stream));
    HIPCHK(c, launch_zero_i32(d.rb_force, nr, c->stream));
    HIPCHK(c, launch_zero_i32(d.rb_any, 2, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)c->md_base, 2 * nr, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.kmax, 2 * nw, c->stream));
    HIPCHK(c, launch_fill_i32((int32_t *)d.lbase, 2 * nw, -1, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.pcount, 2 * nw, c->stream));
    HIPCHK(c, launch_zero_f64(d.wred, 4 * nw, c->stream));
    HIPCHK(c, launch_zero_f64((double *)d.dyn, (int64_t)(sizeof(RepDyn) / 8) * nr, c->stream));
    HIPCHK(c, launch_zero_i32((int32_t *)d.err, 4, c->stream));
    HIPCHK(c, launch_zero_i32(d.counters, 8, c->stream));
    if (d.ring) HIPCHK(c, launch_zero_f64(d.ring, 6 * (int64_t)c->shape.ring, c->stream));
    return KAMD_OK;
}

// Zero the cell counters and the list of the current plan (the counting sort
// expects zero counters; the list kernel overwrites whole rows).
static int init_list(kamd_ctx *c)
{
    Dev &d = c->d;
    HIPCHK(c, launch_zero_i32(d.cell_count, (int64_t)CELL_SUBX * d.ncells, c->stream));
    HIPCHK(c, launch_zero_i32(d.nbr, (int64_t)d.rows * d.npad_total, c->stream));
    return KAMD_OK;
}

// Make the workspace hold `need` bytes with the fixed part preserved.  A
// library-owned workspace is reallocated; a caller-owned one cannot grow
// here: KAMD_ENOMEM, and md_workspace_needed reports the size.
static int grow_workspace(kamd_ctx *c, size_t need)
{
    if (need <= c->ws_bytes) return KAMD_OK;
    c->need_bytes = std::max(c->need_bytes, need);
    if (!c->ws_owned)
        return fail(c, KAMD_ENOMEM, "the caller's workspace of %zu bytes is too small: %zu needed "
                    "(md_workspace_needed, md_set_workspace)", c->ws_bytes, need);
    char *nw = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const hipError_t e = hipMalloc((void **)&nw, need);
    if (e != hipSuccess) return fail(c, KAMD_ENOMEM, "hipMalloc(%zu bytes): %s", need, hipGetErrorString(e));
    HIPCHK(c, hipMemcpyAsync(nw, c->ws, c->list_off, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(c->ws);
    c->ws = nw;
    c->ws_bytes = need;
    return KAMD_OK;
}

static int upload_tables(kamd_ctx *c)
{
    Dev &d = c->d;
    HIPCHK(c, hipMemcpyAsync((void *)d.seg, c->segs.data(), sizeof(SegInfo) * c->segs.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((void *)d.rep, c->rinfo.data(), sizeof(RepInfo) * c->rinfo.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((void *)d.wave_seg, c->wave_seg.data(), 4 * c->wave_seg.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KAMD_OK;
}

static void drop_graph(kamd_ctx *c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_steps = 0;
}

// ---------------------------------------------------------- initial states
// Random sequential addition: uniform proposals, accepted when no placed
// particle is closer than dmin (minimum image); the first n_a accepted are A.
// Falls back to the lattice when the attempt budget runs out.
// dim 2: the plane z = 0 (planar system), with a square cell grid.
static bool rsa_positions(const kamd_replica &K, int dim, double dmin, std::vector<double> &x, std::vector<double> &y,
                          std::vector<double> &z)
{
    const int n = K.n;
    const double L = K.box;
    std::mt19937_64 rng(K.seed ^ 0x5253414b414d4431ull);
    std::uniform_real_distribution<double> U(0.0, L);
    int nc = std::max(1, (int)std::floor(L / dmin));
    if (nc < 3) nc = 1;
    const double cw = L / nc;
    const int ncz = dim == 2 ? 1 : nc;
    std::vector<int> head((size_t)nc * nc * ncz, -1), next(n, -1);
    x.resize(n);
    y.resize(n);
    z.resize(n);
    const double d2 = dmin * dmin;
    int placed = 0;
    const int64_t budget = (int64_t)n * 4000 + 100000;
    int64_t tries = 0;
    auto mi = [L](double d) { if (d > 0.5 * L) d -= L; else if (d < -0.5 * L) d += L; return d; };
    while (placed < n && tries < budget) {
        ++tries;
        double px = U(rng), py = U(rng), pz = dim == 2 ? 0.0 : U(rng);
        int cx = std::min(nc - 1, (int)(px / cw)), cy = std::min(nc - 1, (int)(py / cw)),
            cz = dim == 2 ? 0 : std::min(nc - 1, (int)(pz / cw));
        bool ok = true;
        const int lo = nc >= 3 ? -1 : 0, hi = nc >= 3 ? 1 : 0;
        const int zlo = dim == 2 ? 0 : lo, zhi = dim == 2 ? 0 : hi;
        for (int oz = zlo; oz <= zhi && ok; ++oz)
            for (int oy = lo; oy <= hi && ok; ++oy)
                for (int ox = lo; ox <= hi && ok; ++ox) {
                    int q = (((cz + oz + ncz) % ncz) * nc + (cy + oy + nc) % nc) * nc + (cx + ox + nc) % nc;
                    for (int j = head[q]; j >= 0; j = next[j]) {
                        double dx = mi(px - x[j]), dy = mi(py - y[j]), dz = mi(pz - z[j]);
                        if (dx * dx + dy * dy + dz * dz < d2) { ok = false; break; }
                    }
                }
        if (!ok) continue;
        x[placed] = px;
        y[placed] = py;
        z[placed] = pz;
        int q = (cz * nc + cy) * nc + cx;
        next[placed] = head[q];
        head[q] = placed;
        ++placed;
    }
    return placed == n;
}

// Simple cubic lattice sites (0.5 + k) L/m, then each B particle swaps its
// site with a randomly chosen A particle (Sec. III.A).
// dim 2: a square lattice in the plane z = 0.
static void lattice_positions(const kamd_replica &K, int dim, std::vector<double> &x, std::vector<double> &y,
                              std::vector<double> &z)
{
    const int n = K.n;
    int m = dim == 2 ? (int)std::ceil(std::sqrt((double)n) - 1e-9) : (int)std::ceil(std::cbrt((double)n) - 1e-9);
    while ((dim == 2 ? (int64_t)m * m : (int64_t)m * m * m) < n) ++m;
    const double a = K.box / m;
    x.resize(n);
    y.resize(n);
    z.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = (0.5 + i % m) * a;
        y[i] = (0.5 + (i / m) % m) * a;
        z[i] = dim == 2 ? 0.0 : (0.5 + i / (m * m)) * a;
    }
    std::mt19937_64 rng(K.seed ^ 0x4c41545449434531ull);
    if (K.n_a > 0)
        for (int i = K.n_a; i < n; ++i) {
            std::uniform_int_distribution<int> D(0, K.n_a - 1);
            int j = D(rng);
            std::swap(x[i], x[j]);
            std::swap(y[i], y[j]);
            std::swap(z[i], z[j]);
        }
}

// ---------------------------------------------------------------- kernels
static int rebuild_chain(kamd_ctx *c, const Dev &d)
{
    HIPCHK(c, launch_rb_gate(d, c->stream));
    HIPCHK(c, launch_rb_assign(d, c->stream));
    HIPCHK(c, launch_rb_scan(d, (int)c->segs.size(), c->stream));
    HIPCHK(c, launch_rb_scatter(d, c->stream));
    HIPCHK(c, launch_rb_sortgather(d, c->stream));
    HIPCHK(c, launch_rb_list(d, c->cell_div, c->stream));
    return KAMD_OK;
}

static int force_rebuild_all(kamd_ctx *c)
{
    std::vector<int32_t> ones(c->reps.size(), 1);
    HIPCHK(c, hipMemcpyAsync(c->d.rb_force, ones.data(), 4 * ones.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KAMD_OK;
}

static int forces(kamd_ctx *c, bool energy)
{
    TRY(rebuild_chain(c, c->d));
    HIPCHK(c, launch_force(c->d, c->model, c->cfg.precision, energy, false, c->stream));
    return KAMD_OK;
}

static int mb_reassign(kamd_ctx *c, bool device_tag, uint32_t tag)
{
    const Dev d = c->d;
    if (device_tag) HIPCHK(c, launch_mb_draw_dev(d, c->stream));
    else HIPCHK(c, launch_mb_draw(d, tag, c->stream));
    HIPCHK(c, launch_rep_reduce(d, 7, c->stream));
    HIPCHK(c, launch_mb_center(d, c->stream));
    HIPCHK(c, launch_rep_reduce(d, 1, c->stream));
    HIPCHK(c, launch_mb_scale(d, c->stream));
    return KAMD_OK;
}

static int do_export(kamd_ctx *c)
{
    double *a[9] = {c->st.x, c->st.y, c->st.z, c->st.vx, c->st.vy, c->st.vz, c->st.ax, c->st.ay, c->st.az};
    HIPCHK(c, launch_export(c->d, a, c->st.img, c->stream));
    return KAMD_OK;
}

static int maybe_export(kamd_ctx *c) { return c->cfg.auto_sync ? do_export(c) : KAMD_OK; }

// Whether the observables are sampled at the end of global step gstep.
static bool sample_step(const kamd_ctx *c, int64_t gstep)
{
    return c->d.ring && c->cfg.sample_every > 0 && gstep % c->cfg.sample_every == 0;
}

// Enqueue nsteps steps.  ensemble 0: NVE; 1: NVT with mode/nb/tau.
// device_tags: the Maxwell-Boltzmann draw tags come from the device step
// counter (graph replays), else from the host counter.
static int enqueue_steps(kamd_ctx *c, int nsteps, int ensemble, int mode, int nb, bool device_tags)
{
    const Dev &d = c->d;
    const double dt = c->cfg.dt;
    const int prec = c->cfg.precision;
    if (ensemble == 1 && mode == KAMD_NVT_NOSE_HOOVER) {
        HIPCHK(c, launch_ke_partial(d, c->stream));
        HIPCHK(c, launch_rep_reduce(d, 1, c->stream));
        HIPCHK(c, launch_set_k2(d, c->stream));
        for (int s = 1; s <= nsteps; ++s) {
            const bool smp = sample_step(c, c->step + s);
            HIPCHK(c, launch_nh_begin(d, dt, c->Q_dev, c->stream));
            HIPCHK(c, launch_drift_nh(d, dt, c->stream));
            TRY(rebuild_chain(c, c->d));
            HIPCHK(c, launch_force(d, c->model, prec, smp, true, c->stream));
            HIPCHK(c, launch_kick_nh(d, c->stream));
            HIPCHK(c, launch_rep_reduce(d, smp ? 7 : 1, c->stream));
            HIPCHK(c, launch_nh_end(d, dt, c->Q_dev, c->stream));
            if (smp) HIPCHK(c, launch_sample(d, 7, c->stream));
        }
        return KAMD_OK;
    }
    const bool stoch = ensemble == 1 && mode == KAMD_NVT_STOCHASTIC;
    // The force of a step is fused with its closing half kick and the next
    // drift whenever no thermostat acts in between.  Fused steps alternate
    // the two position mirrors, the two displacement buffers and (FP64) the
    // two packed position buffers; their number is made even so that every
    // call starts and ends on the first buffers (which keeps graph replays
    // consistent).
    std::vector<char> fused(nsteps + 1, 0);
    int nf = 0;
    for (int s = 1; s < nsteps; ++s) {
        const int64_t gstep = c->step + s;
        const bool reassign = stoch && nb > 0 && (gstep % nb) == 0;
        fused[s] = !reassign;
        nf += fused[s];
    }
    if (nf % 2)
        for (int s = 1; s < nsteps; ++s)
            if (fused[s]) { fused[s] = 0; break; }
    uint4 *mir[2] = {c->d.mirror, c->mirror_alt};
    double4 *p4[2] = {c->d.pos4, c->pos4_alt};
    int cur = 0, par = 0;
    Dev dd = c->d;
    bool need_drift = true, p4_ok = false;
    for (int s = 1; s <= nsteps; ++s) {
        dd.mirror = mir[cur];
        dd.maxdisp = c->md_base + par * c->d.nrep;
        dd.pos4 = p4[cur];
        if (need_drift) HIPCHK(c, launch_drift(dd, dt, c->stream));
        TRY(rebuild_chain(c, dd));
        const int64_t gstep = c->step + s;
        const bool reassign = stoch && nb > 0 && (gstep % nb) == 0;
        const bool smp = sample_step(c, gstep);
        if (fused[s]) {
            // the packed positions are current after a fused FP64 step (the
            // list build reorders them with the rest); otherwise pack them
            if (prec == KAMD_PREC_FP64 && !p4_ok) HIPCHK(c, launch_pack_pos(dd, c->stream));
            HIPCHK(c, launch_force_kd(dd, c->model, prec, dt, mir[1 - cur], c->md_base + (1 - par) * c->d.nrep,
                                      p4[1 - cur], smp, c->force_wpb, c->stream));
            if (smp) {
                HIPCHK(c, launch_rep_reduce(dd, 7, c->stream));
                HIPCHK(c, launch_sample(dd, 7, c->stream));
            }
            cur = 1 - cur;
            par = 1 - par;
            need_drift = false;
            p4_ok = true;
            continue;
        }
        p4_ok = false;
        HIPCHK(c, launch_force(dd, c->model, prec, smp, true, c->stream));
        if (s == nsteps || reassign) {
            HIPCHK(c, launch_kick_nve(dd, dt, smp, c->stream));
            if (reassign) {
                // a sample describes the end of the step: PE and W now, KE
                // after the redraw
                if (smp) {
                    HIPCHK(c, launch_rep_reduce(dd, 6, c->stream));
                    HIPCHK(c, launch_sample(dd, 2, c->stream));
                }
                TRY(mb_reassign(c, device_tags, (uint32_t)gstep));
                if (smp) {
                    HIPCHK(c, launch_ke_partial(dd, c->stream));
                    HIPCHK(c, launch_rep_reduce(dd, 1, c->stream));
                    HIPCHK(c, launch_sample(dd, 5, c->stream));
                }
            } else if (smp) {
                HIPCHK(c, launch_rep_reduce(dd, 7, c->stream));
                HIPCHK(c, launch_sample(dd, 7, c->stream));
            }
            need_drift = true;
        } else {
            HIPCHK(c, launch_kick_drift(dd, dt, smp, c->stream));
            if (smp) {
                HIPCHK(c, launch_rep_reduce(dd, 7, c->stream));
                HIPCHK(c, launch_sample(dd, 7, c->stream));
            }
            need_drift = false;
        }
    }
    if (cur != 0 || par != 0) return fail(c, KAMD_EHIP, "internal: unbalanced mirror buffers");
    return KAMD_OK;
}

static int set_Q(kamd_ctx *c, double tau)
{
    std::vector<double> Q(c->reps.size());
    for (size_t r = 0; r < Q.size(); ++r) {
        Q[r] = (double)dim_of(&c->cfg) * c->reps[r].n * c->reps[r].temperature * tau * tau;
        if (!(Q[r] > 0.0)) return fail(c, KAMD_EINVAL, "Nose-Hoover bath mass Q = d N T tau^2 must be > 0 (replica %zu)", r);
    }
    HIPCHK(c, hipMemcpyAsync(c->Q_dev, Q.data(), 8 * Q.size(), hipMemcpyHostToDevice, c->stream));
    return KAMD_OK;
}

static int apply_list_params(kamd_ctx *c, double skin, int cell_div, bool first);

// ---------------------------------------------------- list self-healing
// A neighbour list that outgrows its rows sets KAMD_DEV_LIST_OVERFLOW and
// records in counters[3] the rows its build needed; the force kernels then
// stay inside the truncated list, so that step's forces are wrong.  Eager
// calls check for it before they return: the list gets the rows asked for
// (plus a quarter), and the call's work is redone from the state it started
// from.  Graph replays cannot heal: the bit stays for md_status, and
// md_build_cells then grows the list (the caller recaptures).

// The dynamical state at the start of an eager step call, in caller order.
static int snapshot_save(kamd_ctx *c)
{
    const Dev &d = c->d;
    const size_t nt = d.n_total;
    double *a[9];
    for (int k = 0; k < 9; ++k) a[k] = c->state_tmp + k * nt;
    HIPCHK(c, launch_export(d, a, c->img_tmp, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dyn_snap, d.dyn, sizeof(RepDyn) * c->reps.size(), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->cnt_snap, d.counters, 32, hipMemcpyDeviceToDevice, c->stream));
    return KAMD_OK;
}

static int snapshot_restore(kamd_ctx *c)
{
    const Dev &d = c->d;
    const size_t nt = d.n_total;
    const double *a[9];
    for (int k = 0; k < 9; ++k) a[k] = c->state_tmp + k * nt;
    HIPCHK(c, launch_import(d, a, c->img_tmp, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.dyn, c->dyn_snap, sizeof(RepDyn) * c->reps.size(), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.counters, c->cnt_snap, 32, hipMemcpyDeviceToDevice, c->stream));
    return force_rebuild_all(c);
}

// Waits for the stream.  redo: a list overflowed, the bit is cleared and the
// list has grown to the rows its build asked for.
static int heal_list(kamd_ctx *c, bool &redo)
{
    redo = false;
    uint32_t w = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&w, c->d.err, 4, hipMemcpyDeviceToHost));
    if (!(w & KAMD_DEV_LIST_OVERFLOW)) return KAMD_OK;
    int32_t cnt[8];
    HIPCHK(c, hipMemcpy(cnt, c->d.counters, 32, hipMemcpyDeviceToHost));
    const uint32_t keep = w & ~(uint32_t)KAMD_DEV_LIST_OVERFLOW;
    const int32_t zero = 0;
    HIPCHK(c, hipMemcpy(c->d.err, &keep, 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d.counters + 3, &zero, 4, hipMemcpyHostToDevice));
    const int need = std::max(cnt[3], c->d.rows + 1);
    c->rows_floor = std::max(c->rows_floor, need + need / 4 + LIST_ROW_ALIGN);
    TRY(apply_list_params(c, c->skin, c->cell_div, false));
    redo = true;
    return KAMD_OK;
}

constexpr int HEAL_ATTEMPTS = 4;

// Rebuild the lists (and with `force`, evaluate forces) until no list overflows.
static int heal_build(kamd_ctx *c, bool force, bool energy)
{
    for (int attempt = 0;; ++attempt) {
        if (force) TRY(forces(c, energy));
        else TRY(rebuild_chain(c, c->d));
        bool redo = false;
        TRY(heal_list(c, redo));
        if (!redo) return KAMD_OK;
        if (attempt + 1 >= HEAL_ATTEMPTS)
            return fail(c, KAMD_EDEVICE, "neighbour list still overflows after %d rebuilds", attempt + 1);
    }
}

static int heal_forces(kamd_ctx *c, bool energy) { return heal_build(c, true, energy); }

// Eager steps, redone from the call's starting state while a list overflows.
// On failure (a caller-owned workspace too small for the grown list) the state
// is that of the start of the call.
static int heal_steps(kamd_ctx *c, int nsteps, int ensemble, int mode, int nb)
{
    TRY(snapshot_save(c));
    for (int attempt = 0;; ++attempt) {
        TRY(enqueue_steps(c, nsteps, ensemble, mode, nb, false));
        bool redo = false;
        const int rc = heal_list(c, redo);
        if (rc) {
            (void)snapshot_restore(c);
            return rc;
        }
        if (!redo) return KAMD_OK;
        if (attempt + 1 >= HEAL_ATTEMPTS)
            return fail(c, KAMD_EDEVICE, "neighbour list still overflows after %d rebuilds", attempt + 1);
        TRY(snapshot_restore(c));
    }
}

// ------------------------------------------------------------------ C ABI
extern "C" const char *md_last_error(const kamd_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

namespace kamd {
// For md_init_static: the message md_last_error(NULL) returns after a refusal,
// and the mark that makes md_destroy hand the static array back.
void set_init_error(const char *msg) { g_init_error = msg; }
void mark_static(kamd_ctx *c, int device) { c->static_device = device; }
}  // namespace kamd

// Adopt a skin and cell division (and the list rows of a healed overflow):
// the plan, the tables, and (after md_init) the cell and list part of the
// workspace, which grows when it must.  Forces a full rebuild at the next
// step and drops a captured graph, whose pointers it may invalidate.
static int apply_list_params(kamd_ctx *c, double skin, int cell_div, bool first)
{
    if (!(skin >= 0.0)) return fail(c, KAMD_EINVAL, "skin must be >= 0");
    if (cell_div < 1 || cell_div > 2) return fail(c, KAMD_EINVAL, "cell_div must be 1 or 2");
    Plan P;
    make_plan(&c->cfg, c->reps.data(), (int)c->reps.size(), skin, cell_div, P, c->rows_floor);
    TRY(plan_fits(c, P));
    if (!first) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        TRY(grow_workspace(c, need_for(c, P)));
    }
    c->skin = skin;
    c->cell_div = cell_div;
    c->segs = P.segs;
    c->rinfo = P.rinfo;
    c->wave_seg = P.wave_seg;
    c->plan = P;
    if (!first) {
        drop_graph(c);
        bind_workspace(c, P);
        TRY(init_list(c));
        TRY(upload_tables(c));
        TRY(force_rebuild_all(c));
    }
    return KAMD_OK;
}

extern "C" int md_init(kamd_ctx **out, const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
                       const kamd_state *st, void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!out) return fail(nullptr, KAMD_EINVAL, "out is null");
    *out = nullptr;
    int rc = validate(nullptr, cfg, reps, n_rep);
    if (rc) return rc;
    if (!st) return fail(nullptr, KAMD_EINVAL, "state is null");
    if (cfg->init_mode == KAMD_INIT_GIVEN && (!st->x || !st->y || !st->z || !st->vx || !st->vy || !st->vz))
        return fail(nullptr, KAMD_EINVAL, "KAMD_INIT_GIVEN needs x, y, z, vx, vy, vz");
    if (cfg->init_mode < 0 || cfg->init_mode > 2) return fail(nullptr, KAMD_EINVAL, "bad init_mode");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, KAMD_EHIP, "no HIP device available");
    kamd_ctx *c = new kamd_ctx();
    c->cfg = *cfg;
    c->reps.assign(reps, reps + n_rep);
    c->st = *st;
    c->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&c->device);
    model_from(cfg->model, c->model, c->rc_max);
    if (cfg->pe_unshifted)  // the energy of LAMMPS lj/cut: no V_ab(r_c) term
        for (int p = 0; p < 3; ++p) c->model.vshift[p] = 0.0;
    int r = [&]() -> int {
        TRY(apply_list_params(c, list_skin(cfg), cfg->cell_div <= 0 ? 1 : cfg->cell_div, true));
        const Plan &P = c->plan;
        c->shape = shape_of(cfg, reps, n_rep, P);
        const size_t need = fixed_bytes(c->shape) + list_bytes(P);
        if (workspace) {
            if ((uintptr_t)workspace % 256) return fail(c, KAMD_EINVAL, "workspace must be 256-byte aligned");
            if (ws_bytes < need) {
                c->need_bytes = need;
                return fail(c, KAMD_ENOMEM, "workspace of %zu bytes is too small: md_workspace_size gives %zu",
                            ws_bytes, need);
            }
            c->ws = (char *)workspace;
            c->ws_bytes = ws_bytes;
        } else {
            const hipError_t e = hipMalloc((void **)&c->ws, need);
            if (e != hipSuccess) {
                c->ws = nullptr;
                return fail(c, KAMD_ENOMEM, "hipMalloc(%zu bytes): %s", need, hipGetErrorString(e));
            }
            c->ws_bytes = need;
            c->ws_owned = true;
        }
        bind_workspace(c, P);
        TRY(init_fixed(c));
        TRY(init_list(c));
        TRY(upload_tables(c));
        // slot -> caller index
        std::vector<int32_t> ids(P.npad, -1);
        for (const SegInfo &S : c->segs) {
            const kamd_replica &K = c->reps[S.rep];
            const int64_t first = K.offset + (S.type == 0 ? 0 : K.n_a);
            for (int i = 0; i < S.n; ++i) ids[S.slot0 + i] = (int32_t)(first + i);
        }
        HIPCHK(c, hipMemcpyAsync(c->d.id, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice, c->stream));
        // RDF block table
        for (int q = 0; q < n_rep; ++q)
            for (int i = 0; i < c->reps[q].n; i += BLOCK) {
                c->rdf_block_rep.push_back(q);
                c->rdf_block_start.push_back((int32_t)(c->reps[q].offset + i));
            }
        HIPCHK(c, hipMemcpyAsync((void *)c->d.rdf_block_rep, c->rdf_block_rep.data(), 4 * c->rdf_block_rep.size(),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync((void *)c->d.rdf_block_start, c->rdf_block_start.data(),
                                 4 * c->rdf_block_start.size(), hipMemcpyHostToDevice, c->stream));
        const int64_t nt = P.n_total;
        if (cfg->init_mode == KAMD_INIT_GIVEN) {
            const double *a[9] = {st->x, st->y, st->z, st->vx, st->vy, st->vz, nullptr, nullptr, nullptr};
            HIPCHK(c, launch_import(c->d, a, st->img, c->stream));
        } else {
            std::vector<double> hx(nt), hy(nt), hz(nt);
            // replicas are independent: place them on host threads
            auto place = [&](int q) {
                const kamd_replica &K = c->reps[q];
                std::vector<double> x, y, z;
                bool ok = false;
                const int dm = dim_of(cfg);
                if (cfg->init_mode == KAMD_INIT_RSA) ok = rsa_positions(K, dm, cfg->min_dist > 0 ? cfg->min_dist : 0.8, x, y, z);
                if (!ok) lattice_positions(K, dm, x, y, z);
                std::copy(x.begin(), x.end(), hx.begin() + K.offset);
                std::copy(y.begin(), y.end(), hy.begin() + K.offset);
                std::copy(z.begin(), z.end(), hz.begin() + K.offset);
            };
            const int nthr = std::max(1, std::min<int>(n_rep, (int)std::thread::hardware_concurrency()));
            std::vector<std::thread> pool;
            for (int t = 0; t < nthr; ++t)
                pool.emplace_back([&, t]() {
                    for (int q = t; q < n_rep; q += nthr) place(q);
                });
            for (auto &th : pool) th.join();
            double *tmp = c->state_tmp;  // caller-order staging, 9 n_total doubles
            HIPCHK(c, hipMemcpyAsync(tmp, hx.data(), 8 * nt, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(tmp + nt, hy.data(), 8 * nt, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(tmp + 2 * nt, hz.data(), 8 * nt, hipMemcpyHostToDevice, c->stream));
            const double *a[9] = {tmp, tmp + nt, tmp + 2 * nt, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
            HIPCHK(c, launch_import(c->d, a, nullptr, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            TRY(mb_reassign(c, false, 0u));
        }
        TRY(force_rebuild_all(c));
        TRY(heal_forces(c, false));
        TRY(do_export(c));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return KAMD_OK;
    }();
    if (r) {
        g_init_error = c->err;
        md_destroy(c);
        return r;
    }
    *out = c;
    return KAMD_OK;
}

extern "C" int md_build_cells(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    TRY(force_rebuild_all(c));
    return heal_build(c, false, false);
}

extern "C" int md_forces(kamd_ctx *c, uint32_t flags, double *obs_dev)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    const bool energy = (flags & (KAMD_F_ENERGY | KAMD_F_VIRIAL)) != 0;
    if (energy && !obs_dev) return fail(c, KAMD_EINVAL, "energy/virial requested without obs_dev");
    TRY(heal_forces(c, energy));
    if (energy) {
        HIPCHK(c, launch_rep_reduce(c->d, 6, c->stream));
        HIPCHK(c, launch_store_pe_w(c->d, obs_dev, c->stream));
    }
    return maybe_export(c);
}

extern "C" int md_step_nve(kamd_ctx *c, int32_t nsteps)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (nsteps < 0) return fail(c, KAMD_EINVAL, "nsteps < 0");
    if (nsteps == 0) return KAMD_OK;
    TRY(heal_steps(c, nsteps, 0, 0, 0));
    c->step += nsteps;
    return maybe_export(c);
}

extern "C" int md_step_nvt(kamd_ctx *c, int32_t nsteps, int32_t mode, int32_t n_reassign, double tau)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (nsteps < 0) return fail(c, KAMD_EINVAL, "nsteps < 0");
    if (mode == KAMD_NVT_STOCHASTIC) {
        if (n_reassign <= 0) return fail(c, KAMD_EINVAL, "n_reassign must be > 0");
    } else if (mode == KAMD_NVT_NOSE_HOOVER) {
        if (!(tau > 0.0)) return fail(c, KAMD_EINVAL, "tau must be > 0");
        TRY(set_Q(c, tau));
    } else {
        return fail(c, KAMD_EINVAL, "bad thermostat mode %d", mode);
    }
    if (nsteps == 0) return KAMD_OK;
    TRY(heal_steps(c, nsteps, 1, mode, n_reassign));
    c->step += nsteps;
    return maybe_export(c);
}

extern "C" int md_set_temperature(kamd_ctx *c, const double *temperature)
{
    if (!c || !temperature) return fail(c, KAMD_EINVAL, "null argument");
    for (size_t r = 0; r < c->reps.size(); ++r)
        if (!(temperature[r] > 0.0) || !std::isfinite(temperature[r]))
            return fail(c, KAMD_EINVAL, "temperature of replica %zu must be finite and > 0", r);
    for (size_t r = 0; r < c->reps.size(); ++r) {
        c->reps[r].temperature = temperature[r];
        c->rinfo[r].T = temperature[r];
    }
    HIPCHK(c, hipMemcpyAsync((void *)c->d.rep, c->rinfo.data(), sizeof(RepInfo) * c->rinfo.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KAMD_OK;
}

extern "C" int md_scale_velocities(kamd_ctx *c, const double *factor)
{
    if (!c || !factor) return fail(c, KAMD_EINVAL, "null argument");
    for (size_t r = 0; r < c->reps.size(); ++r)
        if (!(factor[r] >= 0.0) || !std::isfinite(factor[r]))
            return fail(c, KAMD_EINVAL, "velocity factor of replica %zu must be finite and >= 0", r);
    HIPCHK(c, hipMemcpyAsync(c->rep_arg, factor, 8 * c->reps.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_scale_v(c->d, c->rep_arg, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the host array may go away after the call
    return maybe_export(c);
}

extern "C" int md_rdf(kamd_ctx *c, double dr, int32_t n_bins, uint64_t *hist_dev)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (!(dr > 0.0) || !std::isfinite(dr) || n_bins <= 0 || !hist_dev) return fail(c, KAMD_EINVAL, "bad RDF arguments");
    if (3 * (size_t)n_bins * 4 > 60 * 1024) return fail(c, KAMD_EINVAL, "n_bins too large (max 5120)");
    const double rmax = n_bins * dr;
    for (size_t r = 0; r < c->reps.size(); ++r) {
        const double L = c->reps[r].box;
        if (rmax > 0.5 * L * (1.0 + 1e-12))
            return fail(c, KAMD_EINVAL, "n_bins*dr = %.9g exceeds L/2 = %.9g (replica %zu)", rmax, 0.5 * L, r);
    }
    // the grid of each replica is chosen on the device, inside the capacity
    // the workspace holds, so nothing here waits or allocates
    HIPCHK(c, launch_rdf_prepare(c->d, rmax, c->stream));
    HIPCHK(c, launch_rdf(c->d, dr, n_bins, (int)c->rdf_block_rep.size(), hist_dev, c->stream));
    return KAMD_OK;
}

extern "C" int md_msd(kamd_ctx *c, int32_t op, int32_t slot, double *out_dev)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (slot < 0 || slot >= c->d.msd_slots) return fail(c, KAMD_EINVAL, "origin slot must be in [0, %d)", c->d.msd_slots);
    if (op == 0) {
        HIPCHK(c, launch_msd_set(c->d, slot, c->stream));
    } else if (op == 1) {
        if (!out_dev) return fail(c, KAMD_EINVAL, "out_dev is null");
        HIPCHK(c, launch_msd_measure(c->d, slot, c->stream));
        HIPCHK(c, launch_rep_reduce(c->d, 3, c->stream));
        HIPCHK(c, launch_msd_finish(c->d, out_dev, c->stream));
    } else {
        return fail(c, KAMD_EINVAL, "op must be 0 (SET_ORIGIN) or 1 (MEASURE)");
    }
    return KAMD_OK;
}

extern "C" int md_van_hove(kamd_ctx *c, int32_t slot, double dr, int32_t n_bins, uint64_t *hist_dev)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (slot < 0 || slot >= c->d.msd_slots) return fail(c, KAMD_EINVAL, "origin slot must be in [0, %d)", c->d.msd_slots);
    if (!(dr >= 1e-6) || !std::isfinite(dr) || n_bins <= 0 || n_bins > VH_MAX_BINS || !hist_dev)
        return fail(c, KAMD_EINVAL, "bad van Hove arguments (dr >= 1e-6, 0 < n_bins <= %d)", VH_MAX_BINS);
    HIPCHK(c, launch_van_hove(c->d, slot, dr, n_bins, hist_dev, c->stream));
    return KAMD_OK;
}

extern "C" int md_observables(kamd_ctx *c, double *host_out, int32_t max_rows, int32_t *rows)
{
    if (!c || !rows || max_rows < 0 || (max_rows > 0 && !host_out)) return fail(c, KAMD_EINVAL, "bad arguments");
    *rows = 0;
    const Dev &d = c->d;
    if (!d.ring) return KAMD_OK;
    const size_t nr = c->reps.size(), cap = (size_t)d.ring_cap;
    int32_t cnt[8];
    std::vector<double> ring(6 * nr * cap);
    HIPCHK(c, hipMemcpyAsync(cnt, d.counters, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ring.data(), d.ring, 8 * ring.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t total = cnt[2];
    const int64_t k = std::min<int64_t>(std::min<int64_t>(total, (int64_t)cap), max_rows);
    for (size_t r = 0; r < nr; ++r)
        for (int64_t i = 0; i < k; ++i) {
            const size_t slot = (size_t)((total - k + i) % (int64_t)cap);
            std::memcpy(host_out + 6 * (r * (size_t)max_rows + i), &ring[6 * (r * cap + slot)], 6 * sizeof(double));
        }
    *rows = (int32_t)k;
    return KAMD_OK;
}

extern "C" int md_clear_samples(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    HIPCHK(c, launch_zero_i32(c->d.counters + 2, 1, c->stream));
    return KAMD_OK;
}

extern "C" int md_observables_now(kamd_ctx *c, double *host_out)
{
    if (!c || !host_out) return fail(c, KAMD_EINVAL, "null argument");
    const size_t nr = c->reps.size();
    HIPCHK(c, launch_ke_partial(c->d, c->stream));
    HIPCHK(c, launch_rep_reduce(c->d, 1, c->stream));
    HIPCHK(c, launch_store_obs(c->d, c->obs_stage, c->stream));
    std::vector<double> ke(4 * nr), pw(4 * nr);
    HIPCHK(c, hipMemcpyAsync(ke.data(), c->obs_stage, 32 * nr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(heal_forces(c, true));
    HIPCHK(c, launch_rep_reduce(c->d, 6, c->stream));
    HIPCHK(c, launch_store_obs(c->d, c->obs_stage, c->stream));
    HIPCHK(c, hipMemcpyAsync(pw.data(), c->obs_stage, 32 * nr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t r = 0; r < nr; ++r) {
        const double KE = 0.5 * ke[4 * r + 0];
        const double PE = pw[4 * r + 1], W = pw[4 * r + 2];
        const double dd = (double)dim_of(&c->cfg);
        const double n = c->reps[r].n, L = c->reps[r].box, V = dd == 2.0 ? L * L : L * L * L;
        const double T = 2.0 * KE / (dd * n);
        host_out[6 * r + 0] = KE;
        host_out[6 * r + 1] = PE;
        host_out[6 * r + 2] = W;
        host_out[6 * r + 3] = T;
        host_out[6 * r + 4] = KE + PE;
        host_out[6 * r + 5] = n * T / V + W / (dd * V);
    }
    return KAMD_OK;
}

extern "C" int md_thermostat_state(kamd_ctx *c, double *host_out)
{
    if (!c || !host_out) return fail(c, KAMD_EINVAL, "null argument");
    std::vector<RepDyn> dyn(c->reps.size());
    HIPCHK(c, hipMemcpyAsync(dyn.data(), c->d.dyn, sizeof(RepDyn) * dyn.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t r = 0; r < dyn.size(); ++r) {
        host_out[2 * r] = dyn[r].xi;
        host_out[2 * r + 1] = dyn[r].lns;
    }
    return KAMD_OK;
}

extern "C" int md_sync(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    return do_export(c);
}

extern "C" int md_import(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (!c->st.x || !c->st.y || !c->st.z || !c->st.vx || !c->st.vy || !c->st.vz)
        return fail(c, KAMD_EINVAL, "the caller arrays x..vz were not given at md_init");
    const double *a[9] = {c->st.x, c->st.y, c->st.z, c->st.vx, c->st.vy, c->st.vz, nullptr, nullptr, nullptr};
    HIPCHK(c, launch_import(c->d, a, c->st.img, c->stream));
    TRY(force_rebuild_all(c));
    TRY(heal_forces(c, false));
    return maybe_export(c);
}

extern "C" int md_graph_capture(kamd_ctx *c, int32_t nsteps, int32_t ensemble, int32_t mode, int32_t n_reassign,
                                double tau)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (nsteps <= 0) return fail(c, KAMD_EINVAL, "nsteps must be > 0");
    if (ensemble == 1) {
        if (mode == KAMD_NVT_STOCHASTIC) {
            if (n_reassign <= 0 || nsteps % n_reassign) return fail(c, KAMD_EINVAL, "captured stochastic steps need nsteps %% n_reassign == 0");
            if (c->step % n_reassign) return fail(c, KAMD_EINVAL, "capture the stochastic bath at a step count divisible by n_reassign");
        } else if (mode == KAMD_NVT_NOSE_HOOVER) {
            if (!(tau > 0.0)) return fail(c, KAMD_EINVAL, "tau must be > 0");
            TRY(set_Q(c, tau));
        } else {
            return fail(c, KAMD_EINVAL, "bad thermostat mode");
        }
    } else if (ensemble != 0) {
        return fail(c, KAMD_EINVAL, "ensemble must be 0 (NVE) or 1 (NVT)");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    // the device step counter drives the draw tags inside the graph
    int32_t host_step = (int32_t)c->step;
    HIPCHK(c, hipMemcpy(c->d.counters + 1, &host_step, 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int r = enqueue_steps(c, nsteps, ensemble, mode, n_reassign, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(c, KAMD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    c->graph_steps = nsteps;
    return KAMD_OK;
}

extern "C" int md_graph_launch(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (!c->graph_exec) return fail(c, KAMD_ESTATE, "no graph captured");
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    c->step += c->graph_steps;
    return maybe_export(c);
}

extern "C" int md_set_list_params(kamd_ctx *c, double skin, int32_t cell_div)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    return apply_list_params(c, skin, cell_div, false);
}

extern "C" int md_set_force_kernel(kamd_ctx *c, int32_t windows, int32_t wg_size)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (windows != 0 && windows != 1) return fail(c, KAMD_EINVAL, "windows must be 0 or 1");
    if (windows && c->cfg.precision == KAMD_PREC_FP64)
        return fail(c, KAMD_EINVAL, "the FP64 force kernel has no window variant");
    if (wg_size != 0 && wg_size != 64 && wg_size != 128 && wg_size != 256)
        return fail(c, KAMD_EINVAL, "wg_size must be 0, 64, 128 or 256");
    const int wpb = wg_size ? wg_size / WAVE : c->force_wpb;
    if (c->stage_windows == (windows != 0) && c->force_wpb == wpb) return KAMD_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);                  // its launches carry the old kernel and Dev
    c->force_wpb = wpb;
    if (c->stage_windows != (windows != 0)) {
        c->stage_windows = windows != 0;
        c->d.stage_ok = c->cfg.precision != KAMD_PREC_FP64 && c->stage_windows;
        return force_rebuild_all(c);  // the entries change format at the next build
    }
    return KAMD_OK;
}

extern "C" int md_workspace_needed(kamd_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(c, KAMD_EINVAL, "null argument");
    Plan P;
    make_plan(&c->cfg, c->reps.data(), (int)c->reps.size(), c->skin, c->cell_div, P, c->rows_floor);
    *bytes = std::max(c->need_bytes, need_for(c, P));
    return KAMD_OK;
}

extern "C" int md_set_workspace(kamd_ctx *c, void *workspace, size_t ws_bytes)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    if (!workspace || (uintptr_t)workspace % 256) return fail(c, KAMD_EINVAL, "workspace must be non-null and 256-byte aligned");
    if ((char *)workspace == c->ws) return fail(c, KAMD_EINVAL, "that is the current workspace");
    const size_t cur = need_for(c, c->plan);
    if (ws_bytes < cur) {
        c->need_bytes = std::max(c->need_bytes, cur);
        return fail(c, KAMD_ENOMEM, "workspace of %zu bytes is too small: %zu needed", ws_bytes, cur);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the fixed part, the cells and the lists move as they are
    HIPCHK(c, hipMemcpyAsync(workspace, c->ws, cur, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->ws_owned) (void)hipFree(c->ws);
    if (c->static_device >= 0) {  // the device's static array is free for another context
        release_static_workspace(c->static_device);
        c->static_device = -1;
    }
    c->ws = (char *)workspace;
    c->ws_bytes = ws_bytes;
    c->ws_owned = false;
    drop_graph(c);
    bind_workspace(c, c->plan);
    // a list that grew since (a healed overflow) takes its rows now
    if (c->plan.rows < c->rows_floor) TRY(apply_list_params(c, c->skin, c->cell_div, false));
    if (c->need_bytes <= c->ws_bytes) c->need_bytes = 0;
    return KAMD_OK;
}

extern "C" int md_stats(kamd_ctx *c, double *host_out)
{
    if (!c || !host_out) return fail(c, KAMD_EINVAL, "null argument");
    int32_t cnt[8];
    HIPCHK(c, hipMemcpyAsync(cnt, c->d.counters, 32, hipMemcpyDeviceToHost, c->stream));
    std::vector<int32_t> nlen(c->d.npad_total), id(c->d.npad_total);
    std::vector<int2> lb(c->d.nwaves), km(c->d.nwaves);
    HIPCHK(c, hipMemcpyAsync(nlen.data(), c->d.nlen, 4 * nlen.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(id.data(), c->d.id, 4 * id.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(lb.data(), c->d.lbase, sizeof(int2) * lb.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(km.data(), c->d.kmax, sizeof(int2) * km.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t parts_staged = 0;
    for (const int2 &b : lb) parts_staged += (b.x <= -2) + (b.y <= -2);
    // entries every lane of a wavefront walks (its parts padded to the
    // wavefront's longest), summed over the real particles
    double walked = 0.0;
    for (size_t w = 0; w < km.size(); ++w) {
        int real = 0;
        for (int l = 0; l < WAVE; ++l) real += id[w * WAVE + l] >= 0;
        walked += (double)real * (km[w].x + km[w].y);
    }
    double sum = 0.0, mx = 0.0, bytes = 0.0;
    int64_t cntr = 0;
    for (size_t i = 0; i < nlen.size(); ++i)
        if (id[i] >= 0) {
            const int partners = nlen[i] & 0xffff, n16 = (nlen[i] >> 16) & 0xffff;
            sum += partners;
            bytes += 4.0 * (partners - n16) + 2.0 * n16;
            mx = std::max(mx, (double)partners);
            ++cntr;
        }
    host_out[0] = (double)c->step;
    host_out[1] = (double)cnt[0];
    host_out[2] = (double)c->d.n_total;
    host_out[3] = (double)c->d.rows;
    host_out[4] = cntr ? sum / cntr : 0.0;
    host_out[5] = mx;
    host_out[6] = c->skin;
    host_out[7] = (double)c->cell_div;
    host_out[8] = cntr ? bytes / cntr : 0.0;
    host_out[9] = c->d.stage_ok ? 1.0 : 0.0;
    host_out[10] = lb.empty() ? 0.0 : (double)parts_staged / (2.0 * lb.size());
    host_out[11] = (double)(WAVE * c->force_wpb);
    host_out[12] = cntr ? walked / cntr : 0.0;
    double smin = c->skin;
    for (const RepInfo &R : c->plan.rinfo) smin = std::min(smin, R.skin);
    host_out[13] = smin;
    return KAMD_OK;
}

// ------------------------------------------------------------- checkpoints
struct BlobHeader {
    uint64_t magic;
    int64_t n_total;
    int64_t n_rep;
    int64_t step;
};
static const uint64_t BLOB_MAGIC = 0x4b414d4453544131ull;

static size_t blob_size(const kamd_ctx *c)
{
    const size_t nt = c->d.n_total;
    return sizeof(BlobHeader) + 9 * 8 * nt + 3 * 4 * nt + sizeof(RepDyn) * c->reps.size();
}

extern "C" int md_get_state(kamd_ctx *c, void *blob, size_t *bytes)
{
    if (!c || !bytes) return fail(c, KAMD_EINVAL, "null argument");
    const size_t need = blob_size(c);
    if (!blob) { *bytes = need; return KAMD_OK; }
    if (*bytes < need) return fail(c, KAMD_EINVAL, "blob too small (%zu < %zu)", *bytes, need);
    const size_t nt = c->d.n_total;
    double *a[9];
    for (int k = 0; k < 9; ++k) a[k] = c->state_tmp + k * nt;
    HIPCHK(c, launch_export(c->d, a, c->img_tmp, c->stream));
    char *p = (char *)blob;
    BlobHeader h{BLOB_MAGIC, (int64_t)nt, (int64_t)c->reps.size(), c->step};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    HIPCHK(c, hipMemcpyAsync(p, c->state_tmp, 9 * 8 * nt, hipMemcpyDeviceToHost, c->stream));
    p += 9 * 8 * nt;
    HIPCHK(c, hipMemcpyAsync(p, c->img_tmp, 3 * 4 * nt, hipMemcpyDeviceToHost, c->stream));
    p += 3 * 4 * nt;
    HIPCHK(c, hipMemcpyAsync(p, c->d.dyn, sizeof(RepDyn) * c->reps.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return KAMD_OK;
}

extern "C" int md_set_state(kamd_ctx *c, const void *blob, size_t bytes)
{
    if (!c || !blob) return fail(c, KAMD_EINVAL, "null argument");
    if (bytes < blob_size(c)) return fail(c, KAMD_EINVAL, "blob too small");
    BlobHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (h.magic != BLOB_MAGIC || h.n_total != c->d.n_total || h.n_rep != (int64_t)c->reps.size())
        return fail(c, KAMD_EINVAL, "blob does not match this context");
    const size_t nt = c->d.n_total;
    const char *p = (const char *)blob + sizeof h;
    HIPCHK(c, hipMemcpyAsync(c->state_tmp, p, 9 * 8 * nt, hipMemcpyHostToDevice, c->stream));
    p += 9 * 8 * nt;
    HIPCHK(c, hipMemcpyAsync(c->img_tmp, p, 3 * 4 * nt, hipMemcpyHostToDevice, c->stream));
    p += 3 * 4 * nt;
    HIPCHK(c, hipMemcpyAsync(c->d.dyn, p, sizeof(RepDyn) * c->reps.size(), hipMemcpyHostToDevice, c->stream));
    const double *a[9];
    for (int k = 0; k < 9; ++k) a[k] = c->state_tmp + k * nt;
    HIPCHK(c, launch_import(c->d, a, c->img_tmp, c->stream));
    c->step = h.step;
    int32_t host_step = (int32_t)c->step;
    HIPCHK(c, hipMemcpyAsync(c->d.counters + 1, &host_step, 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(force_rebuild_all(c));
    TRY(heal_build(c, false, false));
    return maybe_export(c);
}

extern "C" int md_log_schedule(int32_t n_md, double t0, int32_t kmax, int32_t *out, int32_t max_out, int32_t *count)
{
    if (!count || n_md < 1 || !(t0 >= 0.5) || kmax < 1 || max_out < 0 || (max_out > 0 && !out))
        return fail(nullptr, KAMD_EINVAL, "md_log_schedule: bad argument");
    const double A = std::pow((double)n_md / t0, 1.0 / (double)kmax);
    int32_t n = 0;
    long prev = 0;
    double t = t0;
    for (int guard = 0; guard < 1 << 24; ++guard) {  // A > 1 unless n_md <= t0
        const long s = (long)std::nearbyint(t);
        if (s > n_md) break;
        if (s != prev) {
            if (n < max_out) out[n] = (int32_t)s;
            ++n;
            prev = s;
        }
        if (!(A > 1.0)) break;
        t *= A;
    }
    *count = n;
    return KAMD_OK;
}

extern "C" int md_autotune(kamd_ctx *c, int32_t probe_steps, double *host_out)
{
    if (!c || !host_out) return fail(c, KAMD_EINVAL, "null argument");
    if (probe_steps <= 0) return fail(c, KAMD_EINVAL, "probe_steps must be > 0");
    size_t nb = 0;
    TRY(md_get_state(c, nullptr, &nb));
    std::vector<char> blob(nb);
    TRY(md_get_state(c, blob.data(), &nb));
    const int64_t step0 = c->step;
    const bool mixed = c->cfg.precision != KAMD_PREC_FP64;
    double Lmin = 1e300;
    for (auto &k : c->reps) Lmin = std::min(Lmin, k.box);
    std::vector<double> skins;
    for (double s : {0.2, 0.25, 0.3, 0.35, 0.4, 0.5})
        if (c->rc_max + s < 0.5 * Lmin || s <= 0.2) skins.push_back(s);
    // every candidate must fit the workspace before any is tried
    size_t need = 0;
    for (double s : skins)
        for (int dv = 1; dv <= 2; ++dv) {
            Plan P;
            make_plan(&c->cfg, c->reps.data(), (int)c->reps.size(), s, dv, P, c->rows_floor);
            if (P.ncells_wide <= MAX_PLAN_CELLS) need = std::max(need, need_for(c, P));
        }
    TRY(grow_workspace(c, need));
    struct Cand {
        double skin;
        int div;
        bool win;
        int wpb;
        double ms;
    };
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const int saved_sync = c->cfg.auto_sync;
    const bool win0 = c->stage_windows;
    const int wpb0 = c->force_wpb;
    c->cfg.auto_sync = 0;
    // One candidate from the saved state: a timed warm-up of a quarter of
    // the probe, then the median of three timed runs of probe_steps steps,
    // or of as many as take about 10 ms by the warm-up's rate if that is
    // more (a run must see several list rebuilds, whose cost dominates the
    // differences between candidates of a small system).  A candidate whose
    // list overflows is skipped (ms stays negative).
    auto probe = [&](Cand &k) -> int {
        k.ms = -1.0;
        drop_graph(c);
        c->stage_windows = k.win;
        c->d.stage_ok = mixed && k.win;
        c->force_wpb = k.wpb;
        TRY(apply_list_params(c, k.skin, k.div, false));
        TRY(md_set_state(c, blob.data(), nb));
        const int warm = std::max(1, probe_steps / 4);
        float tw = 0.0f;
        HIPCHK(c, hipEventRecord(e0, c->stream));
        TRY(enqueue_steps(c, warm, 0, 0, 0, false));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&tw, e0, e1));
        const double per = std::max(1e-4, (double)tw / warm);
        const int steps = (int)std::min(20000.0, std::max((double)probe_steps, std::ceil(10.0 / per)));
        float t[3];
        for (int r = 0; r < 3; ++r) {
            HIPCHK(c, hipEventRecord(e0, c->stream));
            TRY(enqueue_steps(c, steps, 0, 0, 0, false));
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            HIPCHK(c, hipEventElapsedTime(&t[r], e0, e1));
        }
        uint32_t word = 0;
        HIPCHK(c, hipMemcpy(&word, c->d.err, 4, hipMemcpyDeviceToHost));
        if (word == 0) {
            std::sort(t, t + 3);
            k.ms = (double)t[1] / steps;
        } else if (word == KAMD_DEV_LIST_OVERFLOW) {  // this candidate's list is too short: skip it
            const uint32_t zero = 0;
            HIPCHK(c, hipMemcpy(c->d.err, &zero, 4, hipMemcpyHostToDevice));
        } else {
            return fail(c, KAMD_EDEVICE, "device error word 0x%x while probing", word);
        }
        return KAMD_OK;
    };
    // Within 1% of the fastest the timings are not told apart reliably; the
    // first such candidate in the order tried is kept.  Stage 1 orders by
    // skin, then grid (the smallest list first); stage 2 tries the direct
    // kernel before the windows, and the larger blocks first.
    auto pick = [](const std::vector<Cand> &v) -> int {
        double fastest = 1e300;
        for (const Cand &k : v)
            if (k.ms > 0.0) fastest = std::min(fastest, k.ms);
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].ms > 0.0 && v[i].ms <= 1.01 * fastest) return (int)i;
        return -1;
    };
    int rc = KAMD_OK;
    // Stage 1: list parameters (skin x cell division) with the current kernel.
    std::vector<Cand> st1;
    for (double s : skins)
        for (int dv = 1; dv <= 2; ++dv) {
            Plan Pt;
            make_plan(&c->cfg, c->reps.data(), (int)c->reps.size(), s, dv, Pt, c->rows_floor);
            if (Pt.ncells_wide <= MAX_PLAN_CELLS) st1.push_back({s, dv, win0, wpb0, -1.0});
        }
    for (Cand &k : st1)
        if (!rc) rc = probe(k);
    const int i1 = rc ? -1 : pick(st1);
    Cand best = i1 >= 0 ? st1[i1] : Cand{c->skin, c->cell_div, win0, wpb0, -1.0};
    // Stage 2: the force kernel at those list parameters: block size
    // {256, 128, 64} threads, and (mixed precisions) windows off or on.
    std::vector<Cand> st2;
    if (i1 >= 0) {
        for (int w = 0; w < (mixed ? 2 : 1); ++w)
            for (int wpb : {4, 2, 1}) {
                if ((w != 0) == best.win && wpb == best.wpb) {
                    st2.push_back(best);  // already timed
                } else {
                    st2.push_back({best.skin, best.div, w != 0, wpb, -1.0});
                    if (!rc) rc = probe(st2.back());
                }
            }
        const int i2 = rc ? -1 : pick(st2);
        if (i2 >= 0) best = st2[i2];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->cfg.auto_sync = saved_sync;
    drop_graph(c);
    c->stage_windows = best.win;
    c->d.stage_ok = mixed && best.win;
    c->force_wpb = best.wpb;
    int rc2 = apply_list_params(c, best.skin, best.div, false);
    if (!rc2) rc2 = md_set_state(c, blob.data(), nb);
    c->step = step0;
    if (rc) return rc;
    if (rc2) return rc2;
    host_out[0] = best.skin;
    host_out[1] = best.div;
    host_out[2] = best.ms;
    host_out[3] = best.win ? 1.0 : 0.0;
    host_out[4] = (double)(best.wpb * WAVE);
    return KAMD_OK;
}

extern "C" int md_profile(kamd_ctx *c, int32_t nsteps, double *host_out)
{
    if (!c || !host_out) return fail(c, KAMD_EINVAL, "null argument");
    if (nsteps <= 0) return fail(c, KAMD_EINVAL, "nsteps must be > 0");
    const double dt = c->cfg.dt;
    const int prec = c->cfg.precision;
    // the same step sequence as md_step_nve, with events around each part
    std::vector<char> fused(nsteps + 1, 0);
    int nf = 0;
    for (int s = 1; s < nsteps; ++s) {
        fused[s] = 1;
        nf += fused[s];
    }
    if (nf % 2)
        for (int s = 1; s < nsteps; ++s)
            if (fused[s]) { fused[s] = 0; break; }
    std::vector<hipEvent_t> ev(5 * (size_t)nsteps + 2);
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    int32_t cnt0[8], cnt1[8];
    HIPCHK(c, hipMemcpyAsync(cnt0, c->d.counters, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint4 *mir[2] = {c->d.mirror, c->mirror_alt};
    double4 *p4[2] = {c->d.pos4, c->pos4_alt};
    int cur = 0, par = 0;
    Dev dd = c->d;
    bool need_drift = true, p4_ok = false;
    size_t k = 0;
    HIPCHK(c, hipEventRecord(ev[k++], c->stream));
    for (int s = 1; s <= nsteps; ++s) {
        dd.mirror = mir[cur];
        dd.maxdisp = c->md_base + par * c->d.nrep;
        dd.pos4 = p4[cur];
        HIPCHK(c, hipEventRecord(ev[k++], c->stream));
        if (need_drift) HIPCHK(c, launch_drift(dd, dt, c->stream));
        HIPCHK(c, hipEventRecord(ev[k++], c->stream));
        TRY(rebuild_chain(c, dd));
        HIPCHK(c, hipEventRecord(ev[k++], c->stream));
        if (fused[s]) {
            if (prec == KAMD_PREC_FP64 && !p4_ok) HIPCHK(c, launch_pack_pos(dd, c->stream));
            HIPCHK(c, launch_force_kd(dd, c->model, prec, dt, mir[1 - cur], c->md_base + (1 - par) * c->d.nrep,
                                      p4[1 - cur], false, c->force_wpb, c->stream));
            cur = 1 - cur;
            par = 1 - par;
            need_drift = false;
            p4_ok = true;
        } else {
            p4_ok = false;
            HIPCHK(c, launch_force(dd, c->model, prec, false, true, c->stream));
        }
        HIPCHK(c, hipEventRecord(ev[k++], c->stream));
        if (!fused[s]) {
            if (s == nsteps) {
                HIPCHK(c, launch_kick_nve(dd, dt, false, c->stream));
            } else {
                HIPCHK(c, launch_kick_drift(dd, dt, false, c->stream));
                need_drift = false;
            }
        }
        HIPCHK(c, hipEventRecord(ev[k++], c->stream));
    }
    HIPCHK(c, hipEventRecord(ev[k++], c->stream));
    HIPCHK(c, hipEventSynchronize(ev[k - 1]));
    double tf = 0.0, ts = 0.0, tr = 0.0;
    float ms = 0.0f;
    for (int s = 0; s < nsteps; ++s) {
        const size_t q = 1 + 5 * (size_t)s;
        HIPCHK(c, hipEventElapsedTime(&ms, ev[q], ev[q + 1])); ts += ms;
        HIPCHK(c, hipEventElapsedTime(&ms, ev[q + 1], ev[q + 2])); tr += ms;
        HIPCHK(c, hipEventElapsedTime(&ms, ev[q + 2], ev[q + 3])); tf += ms;
        HIPCHK(c, hipEventElapsedTime(&ms, ev[q + 3], ev[q + 4])); ts += ms;
    }
    HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[k - 1]));
    const double total = ms;
    for (auto &e : ev) (void)hipEventDestroy(e);
    c->step += nsteps;
    const Dev &d = c->d;
    HIPCHK(c, hipMemcpyAsync(cnt1, d.counters, 32, hipMemcpyDeviceToHost, c->stream));
    // in-cutoff ordered pairs of the final configuration
    TRY(forces(c, true));
    HIPCHK(c, launch_rep_reduce(d, 8, c->stream));
    HIPCHK(c, launch_store_obs(d, c->obs_stage, c->stream));
    std::vector<double> o(4 * c->reps.size());
    HIPCHK(c, hipMemcpyAsync(o.data(), c->obs_stage, 8 * o.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double pairs = 0.0;
    for (size_t r = 0; r < c->reps.size(); ++r) pairs += o[4 * r + 3];
    host_out[0] = tf / nsteps;
    host_out[1] = ts / nsteps;
    host_out[2] = total;
    host_out[3] = (double)(cnt1[0] - cnt0[0]);
    host_out[4] = pairs;
    host_out[5] = nsteps;
    host_out[6] = tr / nsteps;
    host_out[7] = 0.0;
    return maybe_export(c);
}

extern "C" int md_status(kamd_ctx *c, uint32_t *word)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    uint32_t w = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&w, c->d.err, 4, hipMemcpyDeviceToHost));
    if (word) *word = w;
    if (w) return fail(c, KAMD_EDEVICE, "device error word 0x%x", w);
    return KAMD_OK;
}

extern "C" int md_clear_status(kamd_ctx *c)
{
    if (!c) return fail(nullptr, KAMD_EINVAL, "null context");
    const uint32_t zero = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->d.err, &zero, 4, hipMemcpyHostToDevice));
    return KAMD_OK;
}

extern "C" int md_destroy(kamd_ctx *c)
{
    if (!c) return KAMD_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->ws_owned && c->ws) (void)hipFree(c->ws);
    if (c->static_device >= 0) release_static_workspace(c->static_device);
    c->ws = nullptr;
    delete c;
    return KAMD_OK;
}
