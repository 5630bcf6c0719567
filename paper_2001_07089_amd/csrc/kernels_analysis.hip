// kernels_analysis.hip -- on-device radial distribution histogram and
// mean-square displacement.
//
// This translation unit is compiled without floating-point contraction so that
// the pair distance of the histogram is evaluated exactly as the definition
// reads: separations in binary64, minimum image by one +-L correction when
// the separation exceeds L/2 (the branch form of Sec. III.D),
// r^2 = (dx dx + dy dy) + dz dz, r = sqrt(r^2) (IEEE, correctly rounded),
// bin = int(r / dr) by a true division (Sec. VI.A.1).  The counts are then
// identical to those of any other IEEE evaluation of the same definition.
#include "common_dev.hpp"

namespace kamd {

// RDF grid: per replica nc^3 cells (a planar system: one layer of nc^2) of
// edge L/nc >= n_bins*dr, or >= n_bins*dr/2 where such cells still hold
// several particles; both particle types together.  The grid of replica r is
// rdf_grid[r] = {nc, first cell, cells}, chosen on the device (k_rdf_setup),
// so that a measurement needs no host round trip.
// Counting sort into rdf_pos (replica-relative positions, w = type + 2*cell).

// One thread: the grid of every replica for the histogram range r_max.  Cells
// as wide as r_max, or half as wide where such cells would still hold six
// particles or more on average; at most 2 n + 64 cells per replica (wider
// cells stay correct, they only add candidates), so that every grid fits the
// capacity the workspace reserves (2 n_total + 64 n_rep cells).
__global__ void k_rdf_setup(Dev d, double rmax)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const bool planar = d.dim == 2;
    const int cap = planar ? 4096 : 256;
    auto cells = [&](int64_t k) { return planar ? k * k : k * k * k; };
    int cell0 = 0;
    for (int r = 0; r < d.nrep; ++r) {
        const RepInfo &R = d.rep[r];
        const double L = R.L;
        const double hr = 0.5 * rmax;
        const double per_cell = planar ? R.n / (L * L) * (hr * hr) : R.n / (L * L * L) * (hr * hr * hr);
        const double per_range = per_cell >= 6.0 ? 2.0 : 1.0;
        int nc = (int)fmax(1.0, fmin(floor(per_range * L / rmax), (double)cap));
        const int64_t lim = 2 * (int64_t)R.n + 64;
        int nmax = (int)floor(planar ? sqrt((double)lim) : cbrt((double)lim));
        while (cells(nmax + 1) <= lim) ++nmax;
        while (nmax > 1 && cells(nmax) > lim) --nmax;
        nc = max(1, min(nc, nmax));
        d.rdf_grid[r] = make_int4(nc, cell0, (int)cells(nc), 0);
        cell0 += (int)cells(nc);
    }
}

__global__ __launch_bounds__(BLOCK) void k_rdf_assign(Dev d)
{
    const int w = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (w >= d.nwaves) return;
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int s = w * WAVE + lane_id();
    if (s - S.slot0 >= S.n) return;
    const int4 g = d.rdf_grid[S.rep];
    const int nc = g.x;
    const uint4 m = d.mirror[s];
    const int cz = d.dim == 2 ? 0 : fix_cell(m.z, nc);
    const int c = g.y + (cz * nc + fix_cell(m.y, nc)) * nc + fix_cell(m.x, nc);
    d.rdf_cell_of[s] = c;
    d.rdf_rank[s] = atomicAdd(&d.rdf_count[c], 1);
}

// Exclusive scan per replica; rdf_start holds indices into rdf_pos
// (the replica's range begins at its caller offset).
__global__ __launch_bounds__(1024) void k_rdf_scan(Dev d)
{
    __shared__ int part[1024];
    const RepInfo &R = d.rep[blockIdx.x];
    const int4 g = d.rdf_grid[blockIdx.x];
    const int n = g.z;
    const int chunk = (n + 1023) / 1024;
    const int b = threadIdx.x * chunk;
    const int e = min(n, b + chunk);
    int sum = 0;
    for (int c = b; c < e; ++c) sum += d.rdf_count[g.y + c];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = (int)R.caller_off + part[threadIdx.x] - sum;
    for (int c = b; c < e; ++c) {
        d.rdf_start[g.y + c] = run;
        run += d.rdf_count[g.y + c];
    }
}

__global__ __launch_bounds__(BLOCK) void k_rdf_scatter(Dev d)
{
    const int w = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (w >= d.nwaves) return;
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int s = w * WAVE + lane_id();
    if (s - S.slot0 >= S.n) return;
    const int c = d.rdf_cell_of[s];
    const int t = d.rdf_start[c] + d.rdf_rank[s];
    d.rdf_pos[t] = make_double4(d.x[s], d.y[s], d.z[s], (double)(S.type + 2 * (c - d.rdf_grid[S.rep].y)));
}

__device__ inline double min_image_branch(double dd, double L, double half)
{
    if (dd > half) dd -= L;
    else if (dd < -half) dd += L;
    return dd;
}

// One block of BLOCK particles of one replica (block table from the host).
// Each particle visits the distinct cells of its stencil (3 per axis with
// cells as wide as the histogram range r_max, 5 with cells half as wide) that
// come within r_max of it, and counts the partners with a larger index there,
// so every unordered pair is counted once: a partner within range lies in a
// cell within range of both particles, and the one with the smaller index
// counts it.  With the finer cells, leaving out the far ones takes the
// candidates per particle from 27 cells of edge r_max to about 10 of them.
// Block-local u32 histograms in LDS, flushed to the uint64 result.
__device__ inline double cell_gap(int o, int c, double cw, double u)
{
    // distance along one axis from coordinate u (in cell c) to cell c + o
    return o > 0 ? (c + o) * cw - u : (o < 0 ? u - (c + o + 1) * cw : 0.0);
}

__global__ __launch_bounds__(BLOCK) void k_rdf_hist(Dev d, double dr, int nbins, uint64_t *hist)
{
    extern __shared__ uint32_t lh[];  // [3][nbins]
    const int rep = d.rdf_block_rep[blockIdx.x];
    const int i0 = d.rdf_block_start[blockIdx.x];
    const RepInfo &R = d.rep[rep];
    for (int b = threadIdx.x; b < 3 * nbins; b += BLOCK) lh[b] = 0u;
    __syncthreads();
    const int iend = (int)R.caller_off + R.n;
    const int i = i0 + (int)threadIdx.x;
    if (i < iend) {
        const double4 pi = d.rdf_pos[i];
        const int wi = (int)pi.w;
        const int ti = wi & 1;
        const int cl = wi >> 1;
        const int4 g = d.rdf_grid[rep];
        const int nc = g.x;
        const int cx = cl % nc, cy = (cl / nc) % nc, cz = cl / (nc * nc);
        const double L = R.L;
        const double rmax = nbins * dr;
        const int reach = rmax * nc > L * (1.0 + 1e-12) ? 2 : 1;  // cells narrower than r_max
        const int noff = min(nc, 2 * reach + 1);
        const bool whole = nc < 2 * reach + 1;  // every cell along an axis is in the stencil
        const int oz0 = d.dim == 2 ? 0 : -reach, nz = d.dim == 2 ? 1 : noff;  // planar: one layer
        const double half = 0.5 * R.L;
        const double cw = L / nc;
        // pruning radius: the histogram range with a margin far above rounding
        const double rp = rmax * (1.0 + 1e-9) + 1e-12 * L;
        const double rp2 = rp * rp;
        for (int oz = oz0; oz < oz0 + nz; ++oz) {
            const double gz = whole ? 0.0 : cell_gap(oz, cz, cw, pi.z);
            if (gz * gz > rp2) continue;
            const int qz = (cz + oz + 2 * nc) % nc;
            for (int oy = -reach; oy < -reach + noff; ++oy) {
                const double gy = whole ? 0.0 : cell_gap(oy, cy, cw, pi.y);
                const double g2 = gy * gy + gz * gz;
                if (g2 > rp2) continue;
                const int qy = (cy + oy + 2 * nc) % nc;
                for (int ox = -reach; ox < -reach + noff; ++ox) {
                    const double gx = whole ? 0.0 : cell_gap(ox, cx, cw, pi.x);
                    if (gx * gx + g2 > rp2) continue;
                    const int qx = (cx + ox + 2 * nc) % nc;
                    const int c = g.y + (qz * nc + qy) * nc + qx;
                    const int st = d.rdf_start[c];
                    const int en = st + d.rdf_count[c];
                    for (int j = max(st, i + 1); j < en; ++j) {
                        const double4 pj = d.rdf_pos[j];
                        const double dx = min_image_branch(pi.x - pj.x, L, half);
                        const double dy = min_image_branch(pi.y - pj.y, L, half);
                        const double dz = min_image_branch(pi.z - pj.z, L, half);
                        const double r = sqrt(dx * dx + dy * dy + dz * dz);
                        const int bin = (int)(r / dr);
                        if (bin < nbins) {
                            const int p = ti + (((int)pj.w) & 1);
                            atomicAdd(&lh[p * nbins + bin], p == 1 ? 1u : 2u);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    uint64_t *h = hist + (size_t)rep * 3 * nbins;
    for (int b = threadIdx.x; b < 3 * nbins; b += BLOCK)
        if (lh[b]) atomicAdd((unsigned long long *)&h[b], (unsigned long long)lh[b]);
}

// MSD: origin[slot][k][id] = unwrapped coordinate k (x + img L, Sec. VI.B.1).
__global__ __launch_bounds__(BLOCK) void k_msd_set(Dev d, int slot)
{
    const int w = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (w >= d.nwaves) return;
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int s = w * WAVE + lane_id();
    if (s - S.slot0 >= S.n) return;
    const double L = d.rep[S.rep].L;
    const int np = d.npad_total;
    const int g = d.id[s];
    double *o = d.origin + (size_t)slot * 3 * d.n_total;
    o[g] = d.x[s] + (double)d.img[s] * L;
    o[d.n_total + g] = d.y[s] + (double)d.img[np + s] * L;
    o[2 * d.n_total + g] = d.z[s] + (double)d.img[2 * np + s] * L;
}

// Per-wave sum of |r_u - r_u(origin)|^2, stored in component `type` of the
// wave partials (a wave holds one type).
__global__ __launch_bounds__(BLOCK) void k_msd_measure(Dev d, int slot)
{
    const int w = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (w >= d.nwaves) return;
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int s = w * WAVE + lane_id();
    double d2 = 0.0;
    if (s - S.slot0 < S.n) {
        const double L = d.rep[S.rep].L;
        const int np = d.npad_total;
        const int g = d.id[s];
        const double *o = d.origin + (size_t)slot * 3 * d.n_total;
        const double ux = d.x[s] + (double)d.img[s] * L - o[g];
        const double uy = d.y[s] + (double)d.img[np + s] * L - o[d.n_total + g];
        const double uz = d.z[s] + (double)d.img[2 * np + s] * L - o[2 * d.n_total + g];
        d2 = ux * ux + uy * uy + uz * uz;
    }
    d2 = wave_sum(d2);
    if (lane_id() == 0) {
        d.wred[4 * w + 0] = S.type == 0 ? d2 : 0.0;
        d.wred[4 * w + 1] = S.type == 1 ? d2 : 0.0;
    }
}

// Self part of the van Hove function: per replica and species, the histogram
// of |r_u - r_u(origin)| over particles, bin = int(r / dr) kept when
// < n_bins.  Per-wave u32 histograms in LDS (a wave holds one replica and one
// type), flushed to the uint64 result [n_rep][2][n_bins].
__global__ __launch_bounds__(BLOCK) void k_van_hove(Dev d, int slot, double dr, int nbins, uint64_t *hist)
{
    __shared__ uint32_t lh[WAVES_PER_BLOCK][VH_MAX_BINS];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const int w = blockIdx.x * WAVES_PER_BLOCK + wv;
    if (w >= d.nwaves) return;  // per-wave work, no block barrier below
    uint32_t *h = lh[wv];
    for (int b = lane; b < nbins; b += WAVE) h[b] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const SegInfo &S = d.seg[d.wave_seg[w]];
    const int s = w * WAVE + lane;
    if (s - S.slot0 < S.n) {
        const double L = d.rep[S.rep].L;
        const int np = d.npad_total;
        const int g = d.id[s];
        const double *o = d.origin + (size_t)slot * 3 * d.n_total;
        const double dx = d.x[s] + (double)d.img[s] * L - o[g];
        const double dy = d.y[s] + (double)d.img[np + s] * L - o[d.n_total + g];
        const double dz = d.z[s] + (double)d.img[2 * np + s] * L - o[2 * d.n_total + g];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const int bin = (int)(r / dr);
        if (bin < nbins) atomicAdd(&h[bin], 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t *out = hist + ((size_t)S.rep * 2 + S.type) * nbins;
    for (int b = lane; b < nbins; b += WAVE)
        if (h[b]) atomicAdd((unsigned long long *)&out[b], (unsigned long long)h[b]);
}

__global__ void k_msd_finish(Dev d, double *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    const RepInfo &R = d.rep[r];
    out[2 * r + 0] = R.na > 0 ? d.rsum[4 * r + 0] / (double)R.na : 0.0;
    out[2 * r + 1] = R.n - R.na > 0 ? d.rsum[4 * r + 1] / (double)(R.n - R.na) : 0.0;
}

static inline int nblk(const Dev &d) { return (d.nwaves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK; }

hipError_t launch_rdf_prepare(const Dev &d, double rmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_rdf_setup, dim3(1), dim3(64), 0, s, d, rmax);
    hipError_t e = launch_zero_i32(d.rdf_count, d.rdf_cells_cap, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rdf_assign, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    hipLaunchKernelGGL(k_rdf_scan, dim3(d.nrep), dim3(1024), 0, s, d);
    hipLaunchKernelGGL(k_rdf_scatter, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_rdf(const Dev &d, double dr, int nbins, int nblocks, uint64_t *hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_rdf_hist, dim3(nblocks), dim3(BLOCK), sizeof(uint32_t) * 3 * nbins, s, d, dr,
                       nbins, hist);
    return hipGetLastError();
}

hipError_t launch_msd_set(const Dev &d, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_msd_set, dim3(nblk(d)), dim3(BLOCK), 0, s, d, slot);
    return hipGetLastError();
}

hipError_t launch_msd_measure(const Dev &d, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_msd_measure, dim3(nblk(d)), dim3(BLOCK), 0, s, d, slot);
    return hipGetLastError();
}

hipError_t launch_van_hove(const Dev &d, int slot, double dr, int nbins, uint64_t *hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_van_hove, dim3(nblk(d)), dim3(BLOCK), 0, s, d, slot, dr, nbins, hist);
    return hipGetLastError();
}

hipError_t launch_msd_finish(const Dev &d, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_msd_finish, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, out);
    return hipGetLastError();
}

}  // namespace kamd
