// kernels_build.hip -- cell binning, stable counting sort of the internal
// particle order and the neighbour lists.
//
// The paper evaluates forces by a double loop over all pairs and names the
// neighbour list as the optimisation it leaves out (end of Sec. III.E); its
// LAMMPS runs use a binned list with a skin and a rebuild check every step
// (Sec. IV, "neighbor 0.3 bin" with "check yes").  Here each replica has a
// cubic grid of nc^3 cells of edge L/nc >= (largest cutoff + skin)/cell_div
// (a planar system, whose particles all sit at z = 0, a single layer of nc^2),
// and each particle keeps the list of all partners within r_c(ab) + skin,
// rebuilt when some particle of the replica has moved more than skin/2 since
// the last build (so no pair can enter the cutoff unseen).
//
// A rebuild runs as a gate and five (six) kernels, all launched on every
// step, so that the decision stays on the device and the step loop can be
// captured in a HIP graph:
//   rb_gate       one block: rebuild flag of every replica (rebuild_flag),
//                 worklist of the waves of the replicas that rebuild
//   rb_assign     per listed wave: sub-cell index and rank inside the
//                 sub-cell of its particles (one atomic per run of lanes that
//                 share a sub-cell)
//   rb_scan_sum   per chunk of a segment's cells (segments of several chunks
//                 only): the particles of the chunk
//   rb_scan       per chunk: exclusive scan of the counters -> cell ranges
//   rb_scatter    per listed wave: provisional destination slot
//   rb_sortgather per listed particle: its rank by previous slot inside its
//                 sub-cell (a stable sort: the result does not depend on
//                 atomic timing), its state gathered into the scratch
//                 arrays, the counter cleared
//   rb_list       per listed wave: copy its state back, record the build
//                 position, write its neighbour list
// Every kernel returns at once when the worklist is empty; the scan also
// skips replicas whose flag is clear.
#include <climits>

#include "common_dev.hpp"

namespace kamd {

// The gate: one block evaluates the rebuild flag of every replica and writes
// the worklist of the waves of the replicas that rebuild (rb_wlist), replica
// by replica in slot order, with their count in rb_any[0].  On the (most
// frequent) steps without a rebuild every later kernel of the chain exits
// after one load; on a step where a few replicas of a batch rebuild, the
// per-wave kernels spread just their work over the whole device.
constexpr int GATE_THREADS = 1024;
// Replicas come along with those that must rebuild (rebuild_flag) while the
// latter have fewer wavefronts than this: four per SIMD of 256 CUs.
constexpr int LIST_ALONG_WAVES = 4096;

// Rebuild decision of replica r for the running step.  A replica must
// rebuild when forced or when a particle has moved more than half its skin
// since the last build.  On a step where the replicas that must rebuild are
// too few to fill the device (the gate decides, rb_any[1]), the others whose
// largest move has passed REBUILD_ALONG of that come along (`along`): the
// rebuilds of a batch's replicas then fall on fewer steps, whose list builds
// would otherwise each run at the latency of a lone wavefront (an early
// rebuild is always valid).  Every kernel of the rebuild chain evaluates it
// identically: nothing it reads changes before the force kernel of the same
// step closes the check.
constexpr double REBUILD_ALONG = 0.8;
__device__ inline bool rebuild_flag(const Dev &d, int r, bool along)
{
    const double m2 = (double)__uint_as_float(d.maxdisp[r]), t2 = d.rep[r].disp_thr2;
    return d.rb_force[r] != 0 || m2 > t2 || (along && m2 > REBUILD_ALONG * REBUILD_ALONG * t2);
}

// Append, for the replicas of one chunk (one per thread, n of them per
// thread, numbered from first), the numbers first .. first + n - 1 to out,
// in thread order.  Returns the number appended.  Every thread of the block
// calls it.  The threads with n > 0 are compacted first; then the whole block
// writes their ranges with plain stores.
struct GateShared {
    int wtot[GATE_THREADS / WAVE];  // per wavefront: sum of n, then its exclusive prefix
    int wcnt[GATE_THREADS / WAVE];  // per wavefront: threads with n > 0, then their prefix
    int tot, cnt;
    int at[GATE_THREADS], first[GATE_THREADS], n[GATE_THREADS];  // compacted ranges
};

__device__ inline int gate_append(int32_t *out, int n, int first, GateShared &g)
{
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    int inc = n;  // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int u = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += u;
    }
    const uint64_t has = __ballot(n > 0);
    const int rank = __popcll(has & ((1ull << lane) - 1ull));
    if (lane == WAVE - 1) {
        g.wtot[wv] = inc;
        g.wcnt[wv] = __popcll(has);
    }
    __syncthreads();
    if (t == 0) {
        int run = 0, cnt = 0;
        for (int k = 0; k < GATE_THREADS / WAVE; ++k) {
            const int x = g.wtot[k], c = g.wcnt[k];
            g.wtot[k] = run;
            g.wcnt[k] = cnt;
            run += x;
            cnt += c;
        }
        g.tot = run;
        g.cnt = cnt;
    }
    __syncthreads();
    if (n > 0) {
        const int k = g.wcnt[wv] + rank;
        g.at[k] = g.wtot[wv] + inc - n;
        g.first[k] = first;
        g.n[k] = n;
    }
    __syncthreads();
    // The block spreads the output positions, not the ranges: position o
    // belongs to the last range whose start is <= o (the starts ascend, and
    // the first is 0), found by a binary search.
    const int cnt = g.cnt, tot = g.tot;
    for (int o = t; o < tot; o += GATE_THREADS) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.at[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        out[o] = g.first[lo] + (o - g.at[lo]);
    }
    __syncthreads();  // the shared arrays are reused
    return tot;
}

__global__ __launch_bounds__(GATE_THREADS) void k_rb_gate(Dev d)
{
    __shared__ GateShared g;
    __shared__ int wmust;
    // the wavefronts of the replicas that must rebuild; the others come
    // along only while those leave most of the device idle
    if (threadIdx.x == 0) wmust = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < d.nrep; r += GATE_THREADS)
        if (rebuild_flag(d, r, false)) atomicAdd(&wmust, d.rep[r].wave1 - d.rep[r].wave0);
    __syncthreads();
    const int wm = wmust;
    const bool along = wm > 0 && wm < LIST_ALONG_WAVES;
    int nwl = 0;
    for (int r0 = 0; wm > 0 && r0 < d.nrep; r0 += GATE_THREADS) {
        const int r = r0 + threadIdx.x;
        int nw = 0, w0 = 0;
        if (r < d.nrep) {
            const RepInfo &R = d.rep[r];
            w0 = R.wave0;
            if (rebuild_flag(d, r, along)) nw = R.wave1 - R.wave0;
        }
        // most steps rebuild nothing: skip the compaction (block-uniform)
        if (!__syncthreads_or(nw > 0)) continue;
        nwl += gate_append(d.rb_wlist + nwl, nw, w0, g);
    }
    if (threadIdx.x == 0) {
        d.rb_any[0] = nwl;
        d.rb_any[1] = along ? 1 : 0;
    }
}

// Worklist entry of this wavefront for the per-wave kernels that run one
// wave per worklist entry: the first ceil(count / WAVES_PER_BLOCK) blocks
// take part, each XCD a contiguous part of the list; -1 for the rest.
__device__ inline int rb_work_wave(const Dev &d)
{
    const int nact = d.rb_any[0];
    const int nab = (nact + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    if ((int)blockIdx.x >= nab) return -1;
    const int i = xcd_block(blockIdx.x, nab) * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    return i < nact ? d.rb_wlist[i] : -1;
}

// The per-particle kernels of the chain walk the worklist with a grid
// stride over a capped grid (their work per unit is small).
__device__ inline void assign_wave(const Dev &d, int w)
{
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int lane = lane_id();
    const int s = w * WAVE + lane;
    const bool real = (s - S.slot0) < S.n;
    const int nc = d.rep[S.rep].nc;
    int c = -1 - lane;  // distinct dummy for padding lanes
    if (real) {
        const uint4 m = d.mirror[s];
        const int cz = d.dim == 2 ? 0 : fix_cell(m.z, nc);  // planar: one layer of cells
        // sub-cell: the cell, then the quarter of its edge along x
        c = CELL_SUBX * (S.cell0 + (cz * nc + fix_cell(m.y, nc)) * nc) + fix_cell(m.x, CELL_SUBX * nc);
        d.cell_of[s] = c;
    }
    // Runs of consecutive lanes with the same cell (the slots are still in the
    // order of the previous build, so most neighbours share a cell): the first
    // lane of a run reserves the whole run with one atomic.
    const int prev = __shfl_up(c, 1, 64);
    const bool head = (lane == 0) || (prev != c);
    const uint64_t heads = __ballot(head);
    const uint64_t below = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int first = 63 - __clzll((long long)(heads & below));  // head of my run
    const uint64_t above = heads & ~below;
    const int next = above ? __ffsll((long long)above) - 1 : 64;  // head of the next run
    int base = 0;
    if (head && real) base = atomicAdd(&d.cell_count[c], next - lane);
    base = __shfl(base, first, 64);
    if (real) d.rank[s] = base + (lane - first);
}

__global__ __launch_bounds__(BLOCK) void k_rb_assign(Dev d)
{
    const int nact = d.rb_any[0];
    if (nact == 0) return;
    const int stride = gridDim.x * WAVES_PER_BLOCK;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6); i < nact; i += stride)
        assign_wave(d, d.rb_wlist[i]);
}

// Exclusive scan of each segment's sub-cell counters into absolute slot
// ranges [cell_start, cell_end).  A segment's cells come in chunks of
// SCAN_CHUNK (8 consecutive cells per thread of a SCAN_THREADS block; block
// (segment, chunk) of a two-dimensional grid).  A segment of more than one
// chunk first has each chunk's total written by k_rb_scan_sum; k_rb_scan then
// starts each chunk at the segment's first slot plus the totals of the chunks
// before it (at most d.scan_cps - 1 of them), so that the chunks of a large
// system are scanned in parallel instead of one after another.  A cell's
// CELL_SUBX = 4 sub-cell counters are read as one int4 and its ranges written
// as int4s, so a pass moves no more loads and stores than a scan of the cells
// alone would.
static_assert(CELL_SUBX == 4, "the scan reads the sub-cells of a cell as one int4");

__device__ inline int chunk_cells(const SegInfo &S, int c)
{
    return min(S.ncell - c * SCAN_CHUNK, SCAN_CHUNK);
}

constexpr int SCAN_THREADS = SCAN_CHUNK / 8;
constexpr int SCAN_WAVES = SCAN_THREADS / WAVE;

__global__ __launch_bounds__(SCAN_THREADS) void k_rb_scan_sum(Dev d)
{
    __shared__ int wtot[SCAN_WAVES];
    if (d.rb_any[0] == 0) return;
    const SegInfo &S = d.seg[blockIdx.x];
    const int c = blockIdx.y;
    const int n = chunk_cells(S, c);
    if (n <= 0 || !rebuild_flag(d, S.rep, d.rb_any[1] != 0)) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int4 *cnt = reinterpret_cast<const int4 *>(d.cell_count + CELL_SUBX * (S.cell0 + c * SCAN_CHUNK));
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = 8 * t + k;
        if (i < n) {
            const int4 v = cnt[i];
            sum += v.x + v.y + v.z + v.w;
        }
    }
    sum = wave_sum_i(sum);
    if (lane == 0) wtot[wv] = sum;
    __syncthreads();
    if (t == 0) {
        int tot = 0;
        for (int k = 0; k < SCAN_WAVES; ++k) tot += wtot[k];
        d.chunk_sum[blockIdx.x * d.scan_cps + c] = tot;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_rb_scan(Dev d)
{
    __shared__ int wtot[SCAN_WAVES];
    __shared__ int carry_s;
    if (d.rb_any[0] == 0) return;
    const SegInfo &S = d.seg[blockIdx.x];
    const int c = blockIdx.y;
    const int n = chunk_cells(S, c);
    if (n <= 0 || !rebuild_flag(d, S.rep, d.rb_any[1] != 0)) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) {
        int carry = 0;  // the particles of the segment's chunks before this one
        for (int k = 0; k < c; ++k) carry += d.chunk_sum[blockIdx.x * d.scan_cps + k];
        carry_s = carry;
        if (S.type == 0 && c == 0) atomicAdd(&d.counters[0], 1);
    }
    const int4 *cnt = reinterpret_cast<const int4 *>(d.cell_count + CELL_SUBX * (S.cell0 + c * SCAN_CHUNK));
    int4 *cst = reinterpret_cast<int4 *>(d.cell_start + CELL_SUBX * (S.cell0 + c * SCAN_CHUNK));
    int4 *cen = reinterpret_cast<int4 *>(d.cell_end + CELL_SUBX * (S.cell0 + c * SCAN_CHUNK));
    int4 v[8];
    int sum = 0;
    const int i0 = 8 * t;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = (i0 + k < n) ? cnt[i0 + k] : make_int4(0, 0, 0, 0);
        sum += v[k].x + v[k].y + v[k].z + v[k].w;
    }
    int inc = sum;  // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int k = 0; k < SCAN_WAVES; ++k) { const int x = wtot[k]; wtot[k] = run; run += x; }
    }
    __syncthreads();
    int run = S.slot0 + carry_s + wtot[wv] + inc - sum;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (i0 + k < n) {
            int4 a, b;
            a.x = run; run += v[k].x; b.x = run;
            a.y = run; run += v[k].y; b.y = run;
            a.z = run; run += v[k].z; b.z = run;
            a.w = run; run += v[k].w; b.w = run;
            cst[i0 + k] = a;
            cen[i0 + k] = b;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_rb_scatter(Dev d)
{
    const int nact = d.rb_any[0];
    if (nact == 0) return;
    const int stride = gridDim.x * WAVES_PER_BLOCK;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6); i < nact; i += stride) {
        const int w = d.rb_wlist[i];
        const SegInfo &S = d.seg[d.wave_seg[w]];
        const int s = w * WAVE + lane_id();
        if (s - S.slot0 < S.n) d.order[d.cell_start[d.cell_of[s]] + d.rank[s]] = s;
    }
}

// Non-temporal 16-byte store (the build mirror, read once per step).
__device__ inline void st_stream(uint4 v, uint4 *p)
{
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    v4u w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4u *>(p));
}

// One particle's state from slot v to sorted slot t.  The old copy is dead
// once read (non-temporal loads); the sorted copy is read back soon by the
// list builder, and the sorted mirror is its candidates (plain stores).
__device__ inline void gather_one(const Dev &d, int v, int t)
{
    const int np = d.npad_total;
    d.sx[t] = ld_stream(&d.x[v]);
    d.sy[t] = ld_stream(&d.y[v]);
    d.sz[t] = ld_stream(&d.z[v]);
    d.svx[t] = ld_stream(&d.vx[v]);
    d.svy[t] = ld_stream(&d.vy[v]);
    d.svz[t] = ld_stream(&d.vz[v]);
    d.sax[t] = ld_stream(&d.ax[v]);
    d.say[t] = ld_stream(&d.ay[v]);
    d.saz[t] = ld_stream(&d.az[v]);
    d.simg[t] = ld_stream(&d.img[v]);
    d.simg[np + t] = ld_stream(&d.img[np + v]);
    d.simg[2 * np + t] = ld_stream(&d.img[2 * np + v]);
    d.sid[t] = ld_stream(&d.id[v]);
    d.smirror[t] = d.mirror[v];  // the list builder's candidates: cached
}

// One thread per particle of the replicas that rebuild.  The scatter put the
// members of each sub-cell together in `order`, in the order of the atomics
// that counted them; a particle's destination is its sub-cell's start plus
// its rank by previous slot among those members (a loop over the sub-cell, a
// few particles), which makes the counting sort stable.  Each member also
// clears its sub-cell's counter for the next rebuild (a sub-cell without
// members was never counted).
__global__ __launch_bounds__(BLOCK) void k_rb_sortgather(Dev d)
{
    const int nact = d.rb_any[0];
    if (nact == 0) return;
    const int stride = gridDim.x * WAVES_PER_BLOCK;
    for (int i = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6); i < nact; i += stride) {
        const int w = d.rb_wlist[i];
        const SegInfo &S = d.seg[d.wave_seg[w]];
        const int s = w * WAVE + lane_id();
        if (s - S.slot0 < S.n) {
            const int sc = d.cell_of[s];
            const int st = d.cell_start[sc], en = d.cell_end[sc];
            int rank = 0;
            for (int e = st; e < en; ++e) rank += d.order[e] < s ? 1 : 0;
            gather_one(d, s, st + rank);
            d.cell_count[sc] = 0;
        }
    }
}

// Neighbour lists.  One thread per particle.  Entries [0, kA) of a list hold
// the particle's A partners, entries [kA, kA + kB) its B partners, where kA,
// kB are the wavefront maxima rounded up to LIST_ROW_ALIGN.  The part of the
// particle's own type also holds its own slot once (it passes the distance
// test), and unused entries hold it too; the force kernels skip it (zero
// separation).  Storage follows list_index: a particle appends 16 contiguous
// bytes at a time, so cache lines fill completely before they leave the L2.
//
// The stencil is walked row by row: the cells of one stencil row differ only
// in x and are consecutive in the cell-sorted slot order, so a row is one
// contiguous slot range (two when it wraps around the box), scanned eight
// candidates at a time.  With cells as wide as the list radius (reach 1) all
// particles of a cell walk the same 27 cells in the same order, so the lanes
// of a wavefront that share a cell load the same addresses and one cache-line
// access serves all of them; no per-particle pruning is done there, since it
// would break that sharing for little gain.  With finer cells (reach 2) rows,
// and the end cells of a row, that lie farther than the list radius from the
// particle are skipped (in FP64, with a margin), which removes most of the
// 125-cell stencil.  Grids with fewer than 2*reach+1 cells per edge scan
// whole rows.
//
// Candidate test in u32 fixed-point units: the integer difference of two
// coordinates is the minimum-image separation (the box maps onto the full
// 2^32 range), converted to float; rl2_fx is enlarged by a few parts in 10^6
// so that the list is a superset of the exact one.  The sorted mirror has
// LIST_UNROLL spare entries past its end, so the unrolled loads need no clamp.
// Maximum of v over the 64 lanes of a wavefront whose lanes are all active:
// a running maximum along each row of 16 lanes by DPP row shifts (a lane
// with no source lane in its row keeps the identity), then the last lane of
// each row read into a scalar.  A few cycles, where a butterfly of lane
// permutes waits on the LDS crossbar six times.
__device__ inline int wave_max_all(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31);
    const int r2 = __builtin_amdgcn_readlane(v, 47), r3 = __builtin_amdgcn_readlane(v, 63);
    return max(max(r0, r1), max(r2, r3));
}

// Two signed 16-bit lanes of one 32-bit register.
typedef short short2_t __attribute__((ext_vector_type(2)));

// Squared separation minus `bound` (bound >= 1), in units of 2^16 fixed-point
// steps, from coordinates reduced to their high 16 bits: x and y packed in
// one word (x low), z in the low half of another.  Differences wrap modulo
// 2^16, which is the minimum image, as for the full 32-bit coordinates.  The
// x-y sum minus the bound lies in [-bound, 2^31 - bound], so only the final
// sum can saturate, and it does so upwards: the result is negative exactly
// when the squared separation is below the bound.
__device__ inline int r2_coarse_below(uint32_t ixy, uint32_t iz, uint32_t jxy, uint32_t jz, int bound)
{
    const short2_t dxy = __builtin_bit_cast(short2_t, ixy) - __builtin_bit_cast(short2_t, jxy);
    const short2_t dz = __builtin_bit_cast(short2_t, iz) - __builtin_bit_cast(short2_t, jz);
    return __builtin_amdgcn_sdot2(dz, dz, __builtin_amdgcn_sdot2(dxy, dxy, -bound, true), true);
}

__device__ inline double gap(int o, int c, double cw, double u)
{
    return o > 0 ? (c + o) * cw - u : (o < 0 ? u - (c + o + 1) * cw : 0.0);
}

// Accepted entries are staged in LDS, LIST_STAGE per lane, and written out
// four at a time (one 16-byte store per lane) when some lane's stage fills.
// Staging keeps stores out of the scan loop: on this architecture a wait for
// loaded data also waits for every store issued before those loads, so a
// store per candidate batch would expose the store latency on every batch.
//
// Candidate positions are staged too.  With one cell per list radius every
// particle scans, per stencil row, at most two pieces: the main run of cells
// and, where the row wraps around the box, its wrapped end cell.  For each
// piece the wavefront loads the union of its lanes' slot ranges into LDS
// once, with coalesced loads, and the lanes then scan their own ranges out
// of LDS; lanes of one cell read the same LDS words (a broadcast).  A union
// longer than LIST_WIN (lanes in different rows of the grid) is scanned
// straight from global memory instead.
constexpr int LIST_STAGE = 16;
// Boxes up to this edge (in the model's length unit) use the coarse staged
// candidate test; a 2^16-step unit is then at most 0.0034, and the list grows
// by under 0.6%.
constexpr double COARSE_MAX_BOX = 220.0;
constexpr int LIST_WIN = 384;

// STAGE: the window variant of the force kernels is on (d.stage_ok), so
// parts whose windows fit are written in the window format; without it the
// window code is compiled out.
template <bool STAGE>
__global__ __launch_bounds__(BLOCK) void k_rb_list(Dev d, int reach)
{
    __shared__ int32_t stage[WAVES_PER_BLOCK][LIST_STAGE][WAVE];
    __shared__ __attribute__((aligned(16))) uint32_t win_s[WAVES_PER_BLOCK][3][LIST_WIN + LIST_UNROLL];
    if (d.rb_any[0] == 0) return;
    const int w = rb_work_wave(d);  // each XCD walks a contiguous part of the worklist
    if (w < 0) return;
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int rep = S.rep;
    const RepInfo &R = d.rep[rep];
    const int lane = lane_id();
    const int s = w * WAVE + lane;
    const bool real = (s - S.slot0) < S.n;
    const int np = d.npad_total;
    uint4 mi = make_uint4(0, 0, 0, 0);
    double px, py, pz;  // the position, for the FP64 packed copy
    if (real) {
        px = ld_stream(&d.sx[s]);
        py = ld_stream(&d.sy[s]);
        pz = ld_stream(&d.sz[s]);
        st_stream(px, &d.x[s]);
        st_stream(py, &d.y[s]);
        st_stream(pz, &d.z[s]);
        st_stream(ld_stream(&d.svx[s]), &d.vx[s]);
        st_stream(ld_stream(&d.svy[s]), &d.vy[s]);
        st_stream(ld_stream(&d.svz[s]), &d.vz[s]);
        st_stream(ld_stream(&d.sax[s]), &d.ax[s]);
        st_stream(ld_stream(&d.say[s]), &d.ay[s]);
        st_stream(ld_stream(&d.saz[s]), &d.az[s]);
        st_stream(ld_stream(&d.simg[s]), &d.img[s]);
        st_stream(ld_stream(&d.simg[np + s]), &d.img[np + s]);
        st_stream(ld_stream(&d.simg[2 * np + s]), &d.img[2 * np + s]);
        st_stream(ld_stream(&d.sid[s]), &d.id[s]);
        mi = d.smirror[s];
        d.mirror[s] = mi;  // gathered by the next step: cached
        st_stream(mi, &d.mbuild[s]);
    } else {
        px = d.x[s];
        py = d.y[s];
        pz = d.z[s];
    }
    if (d.pos4) d.pos4[s] = make_double4(px, py, pz, 0.0);  // FP64: gathers see the new order
    const int nc = R.nc;
    const int noff = min(nc, 2 * reach + 1);
    const bool whole = nc < 2 * reach + 1;  // every cell of a row is in the stencil
    const bool prune = !whole && reach > 1;
    const int fx = fix_cell(mi.x, CELL_SUBX * nc);  // x in quarter cells
    const int cx = fx / CELL_SUBX, qx = fx % CELL_SUBX;
    const int cy = fix_cell(mi.y, nc), cz = d.dim == 2 ? 0 : fix_cell(mi.z, nc);
    // slot range [cs(c), ce(c)) of cell c (its sub-cells together)
    auto cs = [&](int c) __attribute__((always_inline)) { return d.cell_start[CELL_SUBX * c]; };
    auto ce = [&](int c) __attribute__((always_inline)) { return d.cell_end[CELL_SUBX * c + CELL_SUBX - 1]; };
    // a planar system has every particle in its single (z = 0) layer of cells
    const int oz0 = d.dim == 2 ? 0 : -reach, nz = d.dim == 2 ? 1 : noff;
    const double cw = 4294967296.0 / (double)nc;  // cell edge in fixed units
    const double ux = (double)mi.x, uy = (double)mi.y, uz = (double)mi.z;
    // The staged candidate test compares coordinates reduced to their high
    // 16 bits (x and y packed, z alone) when the box is small enough that the
    // coarse units cost the list almost nothing (below); otherwise full ones.
    const uint32_t ixy = (mi.x >> 16) | (mi.y & 0xffff0000u), iz = mi.z >> 16;
    const bool coarse = R.L <= COARSE_MAX_BOX;
    int32_t *col = d.nbr + list_index(w, d.rows, 0, lane);
    int32_t(*buf)[WAVE] = stage[threadIdx.x / WAVE];
    uint32_t *wx = win_s[threadIdx.x / WAVE][0];
    uint32_t *wy = win_s[threadIdx.x / WAVE][1];
    uint32_t *wz = win_s[threadIdx.x / WAVE][2];
    uint2 *wc = reinterpret_cast<uint2 *>(wx);  // the coarse window: spans wx and wy
    const int rows = d.rows;
    int row = 0;  // 32-bit words of the list used so far
    int total = 0;
    int2 kpart = make_int2(0, 0), bpart = make_int2(-1, -1);  // per part: entries, base
    int2 pcnt = make_int2(0, 0);                              // per part: window pieces (staged)
    int n16 = 0;
    for (int tj = 0; tj < 2; ++tj) {
        const SegInfo &SJ = d.seg[R.seg[tj]];
        const float rl2 = R.rl2_fx[S.type + tj];
        const double rp = sqrt((double)rl2) + 4096.0;  // pruning radius with margin
        // Coarse test.  Truncating both coordinates to 2^16-step units changes
        // their difference by less than one unit per axis, so a pair within
        // the list radius r (in those units) has a coarse separation below
        // r + sqrt(3).  Accepting every coarse r2 below that bound squared
        // keeps the list a superset of the exact one; the extra entries lie
        // in a shell sqrt(3) units thick (0.3% more entries at L = 100).
        const double rc16 = sqrt((double)rl2) * (1.0 / 65536.0) + 1.7320508075688772;
        const int r2c = (int)ceil(rc16 * rc16) + 1;
        const double rp2 = rp * rp;
        // lowest start and highest end of the lanes' non-empty ranges
        // (x = INT_MAX when no lane has one); all lanes take part
        auto span = [&](int st, int en) __attribute__((always_inline)) {
            const bool has = st < en;
            return make_int2(-wave_max_all(has ? -st : INT_MIN + 1), wave_max_all(has ? en : -1));
        };
        // Slot ranges of one stencil row: the main run of cells, and the end
        // cell that wraps around the box where the row does.
        const int32_t *cstart = d.cell_start, *cend = d.cell_end;
        const int cell0 = SJ.cell0;  // kept in a register across the list stores
        auto bounds = [&](int oz, int oy) __attribute__((always_inline)) {
            int4 b = make_int4(0, 0, 0, 0);
            if (real) {
                const int qz = (cz + oz + nc) % nc;
                const int qy = (cy + oy + nc) % nc;
                const int rowc = cell0 + (qz * nc + qy) * nc;  // cell (0, qy, qz)
                if (whole) {
                    b.x = cs(rowc);
                    b.y = ce(rowc + nc - 1);
                } else {
                    // One cell per list radius (reach 1): a particle in
                    // quarter qx of its cell is more than a cell edge, and
                    // so more than the list radius, away along x from the
                    // quarters of the left cell below qx and of the right
                    // cell above qx; both are left out.
                    const int a = cx - reach, e = cx + reach;
                    b.x = cstart[a < 0 ? CELL_SUBX * rowc : CELL_SUBX * (rowc + a) + qx];
                    b.y = cend[e >= nc ? CELL_SUBX * (rowc + nc) - 1 : CELL_SUBX * (rowc + e) + qx];
                    // the left cell wraps to the high end of the row, or
                    // the right cell to its low end
                    const bool lw = a < 0;
                    if (lw || e >= nc) {
                        b.z = cstart[lw ? CELL_SUBX * (rowc + a + nc) + qx : CELL_SUBX * rowc];
                        b.w = cend[lw ? CELL_SUBX * (rowc + nc) - 1 : CELL_SUBX * (rowc + e - nc) + qx];
                    }
                }
            }
            return b;
        };
        // The force kernels' windows (mixed precisions, one cell per list
        // radius).  The part's stencil rows are split into groups, in row
        // order, each as many rows as fit one window: the wavefront's union
        // span of every row piece of the group, one after the other, plus
        // one slot per lane holding that lane's own position.  The force
        // kernel stages and reads one group's window at a time.  Entries of
        // a staged part are 16-bit offsets into their group's window; every
        // lane's entries of a group end at a common count (padding), and
        // the padding points at the lane's own copy (zero separation,
        // skipped like the own slot).  The groups are found in a first pass
        // over the rows, since they decide the format of every entry.
        const int nrow = nz * noff;
        int2 *ptab = d.pieces + ((size_t)w * 2 + tj) * STAGE_PIECES;
        int4 *gtab = d.sgroups + ((size_t)w * 2 + tj) * STAGE_GROUPS;
        int npiece = 0, ngroup = 0, gw = 0, gmax = 0;
        int gw0 = 0, gw1 = 0, gw2 = 0, gw3 = 0;  // window slots of each group (selects, not an array)
        uint32_t gbound = 0;                      // bit r: a new group starts at stencil row r
        const bool try_stage = STAGE && SJ.n > 0 && !prune && nrow <= 32;
        auto close_group = [&]() __attribute__((always_inline)) {
            if (lane == 0 && ngroup < STAGE_GROUPS) gtab[ngroup] = make_int4(npiece, gw, 0, 0);
            gw0 = ngroup == 0 ? gw : gw0;
            gw1 = ngroup == 1 ? gw : gw1;
            gw2 = ngroup == 2 ? gw : gw2;
            gw3 = ngroup == 3 ? gw : gw3;
            gmax = max(gmax, gw);
            ++ngroup;
            gw = 0;
        };
        if (try_stage) {
            int oz = oz0, oy = -reach;
            for (int r = 0; r < nrow; ++r) {
                const int4 b = bounds(oz, oy);
                const int2 p1 = span(b.x, b.y), p2 = span(b.z, b.w);
                const int l1 = p1.x != INT_MAX ? p1.y - p1.x : 0, l2 = p2.x != INT_MAX ? p2.y - p2.x : 0;
                if (gw > 0 && gw + l1 + l2 + WAVE > STAGE_SLOTS) {
                    close_group();
                    gbound |= 1u << r;
                }
                if (l1 > 0) {
                    if (lane == 0 && npiece < STAGE_PIECES) ptab[npiece] = make_int2(p1.x, l1);
                    ++npiece;
                    gw += l1;
                }
                if (l2 > 0) {
                    if (lane == 0 && npiece < STAGE_PIECES) ptab[npiece] = make_int2(p2.x, l2);
                    ++npiece;
                    gw += l2;
                }
                if (++oy == -reach + noff) {
                    oy = -reach;
                    ++oz;
                }
            }
            close_group();
        }
        const bool staged = try_stage && npiece <= STAGE_PIECES && ngroup <= STAGE_GROUPS && gmax + WAVE <= STAGE_SLOTS;
        // Otherwise entries of the part of the particle's own type are stored
        // as 16-bit offsets from a base slot, two to a 32-bit word, when every
        // slot the wavefront can accept (the cell rows of its stencils) and
        // its own slots lie within 2^16 of the lowest of them; else, and for
        // the other part, as 32-bit slot indices.  base = -1 marks 32-bit
        // entries; staged windows use base 0.
        int base = staged ? 0 : -1;
        if (!staged && tj == S.type && SJ.n > 0) {
            int lo = s, hi = s + 1;
            if (real) {
                // lowest and highest stencil row (qz * nc + qy) in slot order;
                // a range that wraps around the box covers both ends
                int z0 = cz + oz0, z1 = cz + oz0 + nz - 1;
                if (z0 < 0 || z1 >= nc) z0 = 0, z1 = nc - 1;
                int y0 = cy - reach, y1 = cy - reach + noff - 1;
                if (y0 < 0 || y1 >= nc) y0 = 0, y1 = nc - 1;
                lo = min(lo, cs(SJ.cell0 + (z0 * nc + y0) * nc));
                hi = max(hi, ce(SJ.cell0 + (z1 * nc + y1) * nc + nc - 1));
            }
            lo = -wave_max_all(-lo);
            hi = wave_max_all(hi);
            if (hi - lo <= 65536) base = lo;
        }
        const bool half = base >= 0;
        const int group = half ? 8 : 4;  // entries per 16-byte store
        auto pack = [&](int a, int b) __attribute__((always_inline)) { return (a - base) | ((b - base) << 16); };
        int cnt = 0;   // entries accepted (and padding between window groups)
        int npad = 0;  // of them padding
        int done = 0;  // entries written to the list (a multiple of group)
        auto flush = [&]() __attribute__((always_inline)) {  // write every complete group of staged entries
            while (done + group <= cnt) {
                const int k = row + (half ? done / 2 : done);  // 32-bit word of the list
                int e[8];
#pragma unroll
                for (int t = 0; t < 4; ++t) e[t] = buf[(done + t) & (LIST_STAGE - 1)][lane];
                if (half) {
#pragma unroll
                    for (int t = 4; t < 8; ++t) e[t] = buf[(done + t) & (LIST_STAGE - 1)][lane];
                }
                const int4 q = half ? make_int4(pack(e[0], e[1]), pack(e[2], e[3]), pack(e[4], e[5]), pack(e[6], e[7]))
                                    : make_int4(e[0], e[1], e[2], e[3]);
                if (k < rows) *reinterpret_cast<int4 *>(col + (k >> 2) * 256) = q;
                done += group;
            }
        };
        // Each candidate is written to the next free stage slot whether or
        // not it is accepted; only an accepted one advances the count.  At
        // the start of a batch at most LIST_STAGE - LIST_UNROLL entries are
        // pending, so the slot written is never one still to be flushed.
        // The particle's own slot passes the test (zero separation) and stays
        // in its list, where the force kernels skip it like the padding.
        // `in` is false only past the end of a range, in the last batch.
        // The entry of slot j is j + dl: dl = 0 for slot indices, the
        // piece's offset in the window minus its first slot when staged.
        int dl = 0;
        auto test = [&](int j, bool in, uint32_t jx, uint32_t jy, uint32_t jz) __attribute__((always_inline)) {
            const float dx = (float)(int)(mi.x - jx);
            const float dy = (float)(int)(mi.y - jy);
            const float dz = (float)(int)(mi.z - jz);
            const float r2 = dx * dx + dy * dy + dz * dz;
            const int acc = (int)in & (int)(r2 < rl2);
            buf[cnt & (LIST_STAGE - 1)][lane] = j + dl;
            cnt += acc;
        };
        auto test_coarse = [&](int j, bool in, uint32_t jxy, uint32_t jz) __attribute__((always_inline)) {
            // the sign bit of r2 - r2c
            const int acc = (int)in & (int)((uint32_t)r2_coarse_below(ixy, iz, jxy, jz, r2c) >> 31);
            buf[cnt & (LIST_STAGE - 1)][lane] = j + dl;
            cnt += acc;
        };
        auto scan = [&](int st, int en) __attribute__((always_inline)) {  // straight from global memory
            int j = st;
            for (; j + LIST_UNROLL <= en; j += LIST_UNROLL) {  // whole batches
                const uint4 *src = d.smirror + j;
                uint4 mj[LIST_UNROLL];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) mj[u] = src[u];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) test(j + u, true, mj[u].x, mj[u].y, mj[u].z);
                if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
            }
            if (j < en) {  // the last, partial batch
                const uint4 *src = d.smirror + j;
                uint4 mj[LIST_UNROLL];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) mj[u] = src[u];
#pragma unroll
                for (int u = 0; u < LIST_UNROLL; ++u) test(j + u, j + u < en, mj[u].x, mj[u].y, mj[u].z);
            }
            if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
        };
        auto scan_staged = [&](int st, int en, int2 sp) __attribute__((always_inline)) {
            const int lo = sp.x, hi = sp.y;
            if (lo == INT_MAX) return;
            if (hi - lo > LIST_WIN) {
                if (st < en) scan(st, en);
                return;
            }
            // up to three loads per lane in flight at once, so that most
            // unions take one memory round trip
            const int n = hi - lo;
            for (int e0 = 0; e0 < n; e0 += 3 * WAVE) {
                uint4 m[3];
#pragma unroll
                for (int t = 0; t < 3; ++t)
                    if (t == 0 || e0 + t * WAVE < n) m[t] = d.smirror[lo + min(e0 + t * WAVE + lane, n - 1)];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int e = e0 + t * WAVE + lane;
                    if (e < n) {
                        if (coarse) {  // (x-y word, z word) pairs: one 8-byte read per candidate
                            wc[e] = make_uint2((m[t].x >> 16) | (m[t].y & 0xffff0000u), m[t].z >> 16);
                        } else {
                            wx[e] = m[t].x;
                            wy[e] = m[t].y;
                            wz[e] = m[t].z;
                        }
                    }
                }
                // No load of this pass is left in flight.  Stated, so that the
                // compiler need not wait for every load (the next row's bounds
                // among them) before it reuses these registers.
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            int j = st;
            if (coarse) {
                for (; j + LIST_UNROLL <= en; j += LIST_UNROLL) {  // whole batches
                    const int o = j - lo;
#pragma unroll
                    for (int u = 0; u < LIST_UNROLL; ++u) test_coarse(j + u, true, wc[o + u].x, wc[o + u].y);
                    if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
                }
                if (j < en) {  // the last, partial batch
                    const int o = j - lo;
#pragma unroll
                    for (int u = 0; u < LIST_UNROLL; ++u) test_coarse(j + u, j + u < en, wc[o + u].x, wc[o + u].y);
                }
            } else {
                for (; j + LIST_UNROLL <= en; j += LIST_UNROLL) {  // whole batches
                    const int o = j - lo;
#pragma unroll
                    for (int u = 0; u < LIST_UNROLL; ++u) test(j + u, true, wx[o + u], wy[o + u], wz[o + u]);
                    if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
                }
                if (j < en) {  // the last, partial batch
                    const int o = j - lo;
#pragma unroll
                    for (int u = 0; u < LIST_UNROLL; ++u) test(j + u, j + u < en, wx[o + u], wy[o + u], wz[o + u]);
                }
            }
            if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        if (SJ.n > 0 && prune) {  // finer cells: per-particle pruning, direct scans
            if (real) {
                for (int oz = oz0; oz < oz0 + nz; ++oz) {
                    const double gz = fmax(gap(oz, cz, cw, uz), 0.0);
                    const int qz = (cz + oz + nc) % nc;
                    for (int oy = -reach; oy < -reach + noff; ++oy) {
                        const double gy = fmax(gap(oy, cy, cw, uy), 0.0);
                        const double g2 = gy * gy + gz * gz;
                        if (g2 > rp2) continue;
                        const int qy = (cy + oy + nc) % nc;
                        const int rowc = SJ.cell0 + (qz * nc + qy) * nc;  // cell (0, qy, qz)
                        int xl = -reach, xr = reach;
                        while (xl < 0) {
                            const double gx = gap(xl, cx, cw, ux);
                            if (gx * gx + g2 <= rp2) break;
                            ++xl;
                        }
                        while (xr > 0) {
                            const double gx = gap(xr, cx, cw, ux);
                            if (gx * gx + g2 <= rp2) break;
                            --xr;
                        }
                        const int a = cx + xl, b = cx + xr;  // unwrapped cell range [a, b]
                        if (a < 0) {
                            scan(cs(rowc + a + nc), ce(rowc + nc - 1));
                            scan(cs(rowc), ce(rowc + b));
                        } else if (b >= nc) {
                            scan(cs(rowc + a), ce(rowc + nc - 1));
                            scan(cs(rowc), ce(rowc + b - nc));
                        } else {
                            scan(cs(rowc + a), ce(rowc + b));
                        }
                    }
                }
            }
        } else if (SJ.n > 0) {  // every lane walks the same rows: staged scans
            // Slot ranges of one stencil row: the main run of cells, and the
            // end cell that wraps around the box where the row does.  Rows
            // are read one step ahead of their scan, so that the loads of a
            // row's bounds overlap the staging loads of the row before.
            int oz = oz0, oy = -reach;
            int4 next = bounds(oz, oy);
            int woff = 0;  // window offset of the next piece (staged)
            int g = 0;     // window group of the row (staged)
            for (int r = 0; r < nrow; ++r) {
                const int4 cur = next;
                const int2 sp1 = span(cur.x, cur.y), sp2 = span(cur.z, cur.w);
                // This row's bounds are used above, before the next row's
                // loads are issued: a wait for them placed after those loads
                // would wait for those loads too.
                __builtin_amdgcn_sched_barrier(0);
                // the next row; after the last one, row 0 again (read, not used)
                if (++oy == -reach + noff) {
                    oy = -reach;
                    if (++oz == oz0 + nz) oz = oz0;
                }
                next = bounds(oz, oy);
                if (staged && ((gbound >> r) & 1u)) {
                    // close group g: every lane's entries up to a common
                    // count (a multiple of the force kernels' 4 entries per
                    // step), padded with its own copy of group g's window
                    const int wg = g == 0 ? gw0 : (g == 1 ? gw1 : (g == 2 ? gw2 : gw3));
                    const int pv = wg + lane;
                    const int kend = (wave_max_all(cnt) + 3) & ~3;
                    while (__any(cnt < kend)) {
                        if (cnt < kend) {
                            buf[cnt & (LIST_STAGE - 1)][lane] = pv;
                            ++cnt;
                            ++npad;
                        }
                        if (__any(cnt - done > LIST_STAGE - LIST_UNROLL)) flush();
                    }
                    if (lane == 0 && g < STAGE_GROUPS) gtab[g].z = kend;
                    ++g;
                    woff = 0;
                }
                if (staged && sp1.x != INT_MAX) {
                    dl = woff - sp1.x;
                    woff += sp1.y - sp1.x;
                }
                scan_staged(cur.x, cur.y, sp1);
                if (staged && sp2.x != INT_MAX) {
                    dl = woff - sp2.x;
                    woff += sp2.y - sp2.x;
                }
                scan_staged(cur.z, cur.w, sp2);
            }
            dl = 0;
        }
        flush();
        total += cnt - npad;
        // padding: the own slot, or in a window the lane's own position copy
        // (of the last group's window)
        const int wlast = ngroup == 1 ? gw0 : (ngroup == 2 ? gw1 : (ngroup == 3 ? gw2 : gw3));
        const int padv = staged ? wlast + lane : s;
        int kmax = wave_max_all(cnt);
        const int align = half ? 2 * LIST_ROW_ALIGN : LIST_ROW_ALIGN;  // whole 16-byte words
        kmax = (kmax + align - 1) / align * align;
        if (done < cnt) {  // the last partial group, padded with the particle's own slot
            const int k = row + (half ? done / 2 : done);
            int e[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) e[t] = done + t < cnt ? buf[(done + t) & (LIST_STAGE - 1)][lane] : padv;
            const int4 q = half ? make_int4(pack(e[0], e[1]), pack(e[2], e[3]), pack(e[4], e[5]), pack(e[6], e[7]))
                                : make_int4(e[0], e[1], e[2], e[3]);
            if (k < rows) *reinterpret_cast<int4 *>(col + (k >> 2) * 256) = q;
            done += group;
        }
        const int words = half ? kmax / 2 : kmax;  // 32-bit words the part occupies
        const int pad = half ? pack(padv, padv) : padv;
        for (int k = row + (half ? done / 2 : done); k < row + words && k < rows; k += 4)
            *reinterpret_cast<int4 *>(col + (k >> 2) * 256) = make_int4(pad, pad, pad, pad);
        if (row + words > rows && lane == 0) set_err(d.err, KAMD_DEV_LIST_OVERFLOW);
        // selects rather than an array indexed by the part, which would
        // live in scratch memory when this loop is not unrolled
        kpart.x = tj == 0 ? kmax : kpart.x;
        kpart.y = tj == 1 ? kmax : kpart.y;
        const int code = staged ? -2 : base;  // -2: entries are offsets into window groups
        bpart.x = tj == 0 ? code : bpart.x;
        bpart.y = tj == 1 ? code : bpart.y;
        pcnt.x = tj == 0 ? (staged ? ngroup : 0) : pcnt.x;
        pcnt.y = tj == 1 ? (staged ? ngroup : 0) : pcnt.y;
        if (half) n16 += cnt - npad - (tj == S.type ? 1 : 0);  // 16-bit partner entries (not the own slot)
        row += words;
    }
    if (row > rows) {  // keep the force kernels inside the list
        if (lane == 0) atomicMax(&d.counters[3], row);  // the rows a healing rebuild must provide
        const bool h0 = bpart.x >= 0 || bpart.x <= -2, h1 = bpart.y >= 0 || bpart.y <= -2;  // 16-bit parts
        const int w0 = min(h0 ? kpart.x / 2 : kpart.x, rows);
        const int w1 = min(h1 ? kpart.y / 2 : kpart.y, rows - w0);
        kpart.x = h0 ? 2 * w0 : w0;
        kpart.y = h1 ? 2 * w1 : w1;
    }
    if (lane == 0) {
        d.kmax[w] = kpart;
        d.lbase[w] = bpart;
        d.pcount[w] = pcnt;
    }
    // partners (without the own slot) in the low 16 bits, those of them
    // stored as 16-bit entries in the high 16 bits
    d.nlen[s] = real ? (total - 1) | (n16 << 16) : 0;
}

static inline int nblk_slots(const Dev &d) { return (d.nwaves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK; }
constexpr int CHAIN_MAX_BLOCKS = 1024;  // grid cap of the grid-stride chain kernels
static inline int nblk_capped(int waves) { return std::min((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK, CHAIN_MAX_BLOCKS); }

hipError_t launch_rb_gate(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rb_gate, dim3(1), dim3(GATE_THREADS), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_rb_assign(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rb_assign, dim3(nblk_capped(d.nwaves)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_rb_scan(const Dev &d, int nseg, hipStream_t s)
{
    const dim3 grid(nseg, d.scan_cps);
    if (d.scan_cps > 1) hipLaunchKernelGGL(k_rb_scan_sum, grid, dim3(SCAN_THREADS), 0, s, d);
    hipLaunchKernelGGL(k_rb_scan, grid, dim3(SCAN_THREADS), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_rb_scatter(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rb_scatter, dim3(nblk_capped(d.nwaves)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_rb_sortgather(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rb_sortgather, dim3(nblk_capped(d.nwaves)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_rb_list(const Dev &d, int cell_div, hipStream_t s)
{
    if (d.stage_ok)
        hipLaunchKernelGGL(k_rb_list<true>, dim3(nblk_slots(d)), dim3(BLOCK), 0, s, d, cell_div);
    else
        hipLaunchKernelGGL(k_rb_list<false>, dim3(nblk_slots(d)), dim3(BLOCK), 0, s, d, cell_div);
    return hipGetLastError();
}

}  // namespace kamd
