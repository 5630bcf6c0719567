// kernels_force.hip -- Kob-Andersen pair forces over the neighbour lists.
//
// Force on particle i, Eq. (KAFix): F_i = 48 sum_j eps_ab (sig_ab^12/r^14 -
// 0.5 sig_ab^6/r^8)(r_i - r_j) over partners with r < 2.5 sig_ab (strict),
// computed as 48 eps * s6 (s6 - 1/2) / r^2 with s6 = (sig^2/r^2)^3 so that no
// square root is needed and the factor 48 eps is applied once per partner
// type (the paper's own two savings, Sec. III.D).  With the energy flag the
// shifted potential of Eq. (VshiftedKALJ), 4 eps s6 (s6 - 1) - V(r_c), and the
// virial r.F = 48 eps s6 (s6 - 1/2) are accumulated too (each pair appears in
// both partners' lists, so the per-particle sums are halved), together with
// the number of (ordered) pairs inside the cutoff.
//
// One thread per particle; a wavefront holds 64 particles of one replica and
// one type, so the parameters of each list part (A partners, then B partners,
// the paper's type-split loops) are wavefront-uniform and live in scalar
// registers.  Work is plain vector ALU arithmetic: a pair force is not a dense
// contraction, so there is nothing for the matrix cores here.
//
// Precision variants (template PREC):
//   0  FP64: binary64 separations with the minimum image taken as
//      d - L rint(d/L), binary64 LJ terms and sums.
//   1  MIXED: the separation is the exact integer difference of u32
//      fixed-point coordinates (minimum image for free), converted to FP32;
//      FP32 r^2, 1/r^2, LJ terms and per-part partial sums; the part sums are
//      scaled to force units and added in FP64.
//   2  MIXED_FIXED: as MIXED, but every pair force component is rounded to an
//      integer number of 2^-26 force units (one FP64 fma against 1.5*2^52)
//      and summed in 64-bit integers, so the sum is exact and independent of
//      the order of the list; F_ij = -F_ji holds bit for bit.  The rounding
//      is exact only while |F| < 2^25 per pair: each list part tracks its
//      largest in-cutoff 1/r^2 and the kernel sets KAMD_DEV_FORCE_RANGE when
//      a pair came closer than the separation where that bound is reached.
#include "common_dev.hpp"

namespace kamd {

// Close the rebuild check of the running step (every kernel of the rebuild
// chain has finished reading it) and optionally advance the device step
// counter.  Done by the first block of every force launch.
__device__ inline void close_step(const Dev &d, int step_inc)
{
    if (blockIdx.x != 0) return;
    for (int r = threadIdx.x; r < d.nrep; r += blockDim.x) {
        d.maxdisp[r] = 0u;
        d.rb_force[r] = 0;
    }
    if (step_inc && threadIdx.x == 0) d.counters[1] += 1;
}

__device__ inline double rcp_f64(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

// Entries k .. k+3 of a list part (k a multiple of 4).  32-bit entries fill
// a 16-byte word.  16-bit entries (offsets from base) fill half of one, and
// the next four are the other half of the same word (a cache hit), so that
// both formats gather four neighbours per pass.
__device__ inline void list_quad32(const int4 *nb, int k, int jj[4])
{
    const int4 q = ld_stream(nb + (k >> 2) * WAVE);  // read once per step
    jj[0] = q.x;
    jj[1] = q.y;
    jj[2] = q.z;
    jj[3] = q.w;
}
__device__ inline void list_quad16(const int4 *nb, int k, int base, int jj[4])
{
    const int4 q = nb[(k >> 3) * WAVE];
    const bool hi = (k & 4) != 0;
    const uint32_t a = (uint32_t)(hi ? q.z : q.x), b = (uint32_t)(hi ? q.w : q.y);
    jj[0] = base + (int)(a & 0xffffu);
    jj[1] = base + (int)(a >> 16);
    jj[2] = base + (int)(b & 0xffffu);
    jj[3] = base + (int)(b >> 16);
}

// FP64 positions of every slot packed as (x, y, z, 0), so that the FP64 force
// kernel gathers a neighbour with two 16-byte loads instead of three 8-byte
// ones: the gathers bound that kernel, and their cost is per instruction.
__global__ __launch_bounds__(BLOCK) void k_pack_pos(Dev d)
{
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s < d.npad_total) d.pos4[s] = make_double4(d.x[s], d.y[s], d.z[s], 0.0);
}

// KD (NVE steps only): as in the mixed kernel below, the force of slot s
// closes the step's half kick and opens the next one (drift, wrap, new
// mirror into mirror_out, displacement into md_out).  Neighbours gather from
// d.pos4, so the new positions go to d.x, d.y, d.z in place and, packed, to
// pos4_out (a different buffer), where the next step's neighbours find them.
// Padding slots copy their unchanged position, which keeps their own list
// entry at zero separation.
template <bool ENERGY, bool KD, int WPB>
__global__ __launch_bounds__(WAVE * WPB) void k_force_fp64(Dev d, Model m, int step_inc, double dt,
                                                            uint4 *mirror_out, uint32_t *md_out, double4 *pos4_out)
{
    close_step(d, step_inc);
    const int w = wave_id_remapped<WPB>();
    const bool valid = w < d.nwaves;
    float d2 = 0.0f;
    int rep = -1;
    if (valid) {
    const SegInfo &S = d.seg[d.wave_seg[w]];
    rep = S.rep;
    const RepInfo &R = d.rep[S.rep];
    const int s = w * WAVE + lane_id();
    const double L = R.L, invL = R.invL;
    const double xi = d.x[s], yi = d.y[s], zi = d.z[s];
    const int2 km = d.kmax[w];
    const int2 lb = d.lbase[w];
    double fx = 0.0, fy = 0.0, fz = 0.0, pe = 0.0, vir = 0.0, npair = 0.0, ke2 = 0.0;
    int row = 0;  // 32-bit words of the list
#pragma unroll 1
    for (int tj = 0; tj < 2; ++tj) {
        const int p = S.type + tj;
        const double rc2 = m.rc2[p], sig2 = m.sig2[p];
        const int nrows = tj ? km.y : km.x;
        const int base = tj ? lb.y : lb.x;
        double sx = 0.0, sy = 0.0, sz = 0.0, se = 0.0, sv = 0.0;
        int cnt = 0;
        const int4 *nb = reinterpret_cast<const int4 *>(d.nbr + list_index(w, d.rows, row, lane_id()));
        auto pair = [&](double xj, double yj, double zj) {
                double dx = xi - xj;
                double dy = yi - yj;
                double dz = zi - zj;
                dx = fma(-L, rint(dx * invL), dx);
                dy = fma(-L, rint(dy * invL), dy);
                dz = fma(-L, rint(dz * invL), dz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const bool in = (r2 < rc2) && (r2 > 0.0);
                const double ir2 = in ? rcp_f64(r2) : 0.0;
                const double s2 = sig2 * ir2;
                const double s6 = s2 * s2 * s2;
                const double t = s6 * (s6 - 0.5);
                const double f = t * ir2;
                sx = fma(f, dx, sx);
                sy = fma(f, dy, sy);
                sz = fma(f, dz, sz);
                if (ENERGY) {
                    se += fma(-0.5, s6, t);
                    sv += t;
                    cnt += in ? 1 : 0;
                }
        };
        auto quad = [&](const int jj[4]) {
            double4 pj[4];  // two 16-byte loads per neighbour instead of three 8-byte ones
#pragma unroll
            for (int u = 0; u < 4; ++u) pj[u] = d.pos4[jj[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) pair(pj[u].x, pj[u].y, pj[u].z);
        };
        if (base <= -2) {  // a window list is never built for FP64
            if (lane_id() == 0) set_err(d.err, KAMD_DEV_LIST_FORMAT);
        } else if (base >= 0) {
            for (int k = 0; k < nrows; k += 4) {
                int jj[4];
                list_quad16(nb, k, base, jj);
                quad(jj);
            }
        } else {
            for (int k = 0; k < nrows; k += 4) {
                int jj[4];
                list_quad32(nb, k, jj);
                quad(jj);
            }
        }
        const double e48 = 48.0 * m.eps[p];
        fx = fma(e48, sx, fx);
        fy = fma(e48, sy, fy);
        fz = fma(e48, sz, fz);
        if (ENERGY) {
            pe += 0.5 * (4.0 * m.eps[p] * se - (double)cnt * m.vshift[p]);
            vir += 0.5 * e48 * sv;
            npair += (double)cnt;
        }
        row += base >= 0 ? nrows / 2 : nrows;
    }
    if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) set_err(d.err, KAMD_DEV_NONFINITE);
    if (!KD) {
        d.ax[s] = fx;
        d.ay[s] = fy;
        d.az[s] = fz;
    } else if ((s - S.slot0) < S.n) {
        const double h = 0.5 * dt;
        const double a[3] = {fx, fy, fz};
        const double v[3] = {fma(h, fx, ld_stream(&d.vx[s])), fma(h, fy, ld_stream(&d.vy[s])), fma(h, fz, ld_stream(&d.vz[s]))};
        if (ENERGY) ke2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        drift_core(d, s, R, dt, 0.0, 0.0, h, v, a, mirror_out, d2);
        pos4_out[s] = make_double4(d.x[s], d.y[s], d.z[s], 0.0);
    } else {
        pos4_out[s] = make_double4(xi, yi, zi, 0.0);
    }
    if (ENERGY) {
        pe = wave_sum(pe);
        vir = wave_sum(vir);
        npair = wave_sum(npair);
        if (KD) ke2 = wave_sum(ke2);
        if (lane_id() == 0) {
            if (KD) d.wred[4 * w + 0] = ke2;
            d.wred[4 * w + 1] = pe;
            d.wred[4 * w + 2] = vir;
            d.wred[4 * w + 3] = npair;
        }
    }
    }
    if (KD) block_disp_max<WPB>(md_out, valid, rep, d2);
}

// LDS visible to the whole wavefront (the lanes wrote it, others read it).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// KD (NVE steps only): after the force of slot s, close the step with the
// half kick v += a dt/2 and open the next one (v += a dt/2, r += v dt, wrap,
// new mirror into mirror_out, displacement into md_out) in the same pass.
// Neighbours read their positions from d.mirror while mirror_out receives the
// new ones, so the two must be different buffers; the forces are not stored.
//
// STAGE: a list part whose windows fit (lbase = -2, written by the list
// builder) is gathered from LDS.  Its stencil rows come in up to STAGE_GROUPS
// groups; for each group the wavefront copies the slot ranges of the group's
// row pieces (its lanes' union span of each stencil row, coalesced loads of
// d.mirror) one after the other into its window, and each lane its own
// position after them, then reads the group's entries, 16-bit offsets into
// that window.  A gather from global memory costs the kernel one cache-line
// access per lane and waits on the vector L1; a window read does neither.
// Parts whose windows do not fit keep the slot-index entries.
// Wavefronts per SIMD the register allocation of the staged step variant
// must allow: its LDS allows 5 (four wavefronts per block), and unbounded it
// takes a few registers too many for that (two 8-byte values then live in
// scratch, stored once per wavefront).
constexpr int WPE_STAGED = 5;

template <bool FIXED, bool ENERGY, bool KD, bool STAGE, int WPB>
__global__ __launch_bounds__(WAVE * WPB) __attribute__((amdgpu_waves_per_eu(STAGE && !ENERGY ? WPE_STAGED : 1))) void k_force_mixed(Dev d, Model m, int step_inc, double dt,
                                                             uint4 *mirror_out, uint32_t *md_out)
{
    __shared__ uint32_t swin[STAGE ? WPB : 1][STAGE ? 3 * STAGE_SLOTS : 1];
    close_step(d, step_inc);
    const int w = wave_id_remapped<WPB>();
    const bool valid = w < d.nwaves;
    float d2 = 0.0f;
    int rep = -1;
    if (valid) {
    const SegInfo &S = d.seg[d.wave_seg[w]];
    rep = S.rep;
    const RepInfo &R = d.rep[S.rep];
    const int s = w * WAVE + lane_id();
    const uint4 mi = d.mirror[s];
    const int2 km = d.kmax[w];
    const int2 lb = d.lbase[w];
    const int2 pc = STAGE ? d.pcount[w] : make_int2(0, 0);
    uint32_t *win = swin[STAGE ? threadIdx.x >> 6 : 0];
    double fx = 0.0, fy = 0.0, fz = 0.0, pe = 0.0, vir = 0.0, npair = 0.0, ke2 = 0.0;
    uint64_t qx = 0, qy = 0, qz = 0;
    bool range_bad = false;
    int row = 0;  // 32-bit words of the list
#pragma unroll 1
    for (int tj = 0; tj < 2; ++tj) {
        const int p = S.type + tj;
        const float rc2 = R.rc2_fx[p], sig2 = R.sig2_fx[p];
        const double fk = R.fix_k[p];
        const int nrows = tj ? km.y : km.x;
        const int base = tj ? lb.y : lb.x;
        float sx = 0.0f, sy = 0.0f, sz = 0.0f, se = 0.0f, sv = 0.0f;
        float irmax = 0.0f;  // largest 1/r^2 of an in-cutoff pair (fixed-point range check)
        int cnt = 0;
        const int4 *nb = reinterpret_cast<const int4 *>(d.nbr + list_index(w, d.rows, row, lane_id()));
        auto pair = [&](const uint4 mj) {
                const int ix = (int)(mi.x - mj.x);
                const int iy = (int)(mi.y - mj.y);
                const int iz = (int)(mi.z - mj.z);
                const float dx = (float)ix, dy = (float)iy, dz = (float)iz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool in = (r2 < rc2) && (r2 > 0.0f);
                const float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
                const float s2 = sig2 * ir2;
                const float s6 = s2 * s2 * s2;
                const float t = s6 * (s6 - 0.5f);
                const float f = t * ir2;
                if (FIXED) {
                    irmax = fmaxf(irmax, ir2);
                    const double wd = (double)f * fk;
                    qx += (uint64_t)__double_as_longlong(fma(wd, (double)ix, FIX_MAGIC));
                    qy += (uint64_t)__double_as_longlong(fma(wd, (double)iy, FIX_MAGIC));
                    qz += (uint64_t)__double_as_longlong(fma(wd, (double)iz, FIX_MAGIC));
                } else {
                    sx = fmaf(f, dx, sx);
                    sy = fmaf(f, dy, sy);
                    sz = fmaf(f, dz, sz);
                }
                if (ENERGY) {
                    se += fmaf(-0.5f, s6, t);
                    sv += t;
                    cnt += in ? 1 : 0;
                }
        };
        auto quad = [&](const int jj[4]) {
            uint4 mj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) mj[u] = d.mirror[jj[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) pair(mj[u]);
        };
        if (!STAGE && base <= -2) {  // a window list for the direct variant: never read it as slots
            if (lane_id() == 0) set_err(d.err, KAMD_DEV_LIST_FORMAT);
        } else if (STAGE && base <= -2) {
            const int ng = tj ? pc.y : pc.x;
            const int2 *pt = d.pieces + ((size_t)w * 2 + tj) * STAGE_PIECES;
            const int4 *gt = d.sgroups + ((size_t)w * 2 + tj) * STAGE_GROUPS;
            int q = 0, k = 0;
            for (int g = 0; g < ng; ++g) {
                const int4 gi = gt[g];  // (end of its pieces, window slots, end of its entries, -)
                const int kend = min(g + 1 < ng ? gi.z : nrows, nrows);
                int off = 0;
                for (; q < gi.x; ++q) {
                    const int2 pq = pt[q];
                    // two loads in flight per lane before the first store
                    for (int e = lane_id(); e < pq.y; e += 2 * WAVE) {
                        const bool two = e + WAVE < pq.y;
                        const uint4 ma = d.mirror[pq.x + e];
                        const uint4 mb = d.mirror[pq.x + (two ? e + WAVE : e)];
                        uint32_t *o = win + 3 * (off + e);
                        o[0] = ma.x;
                        o[1] = ma.y;
                        o[2] = ma.z;
                        if (two) {
                            o[3 * WAVE + 0] = mb.x;
                            o[3 * WAVE + 1] = mb.y;
                            o[3 * WAVE + 2] = mb.z;
                        }
                    }
                    off += pq.y;
                }
                uint32_t *o = win + 3 * (gi.y + lane_id());
                o[0] = mi.x;
                o[1] = mi.y;
                o[2] = mi.z;
                wave_lds_sync();
                for (; k < kend; k += 4) {
                    int jj[4];
                    list_quad16(nb, k, 0, jj);
                    uint4 mj[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t *src = win + 3 * jj[u];
                        mj[u] = make_uint4(src[0], src[1], src[2], 0u);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) pair(mj[u]);
                }
                wave_lds_sync();  // the next group (or part) stages over this window
            }
        } else if (base >= 0) {
            for (int k = 0; k < nrows; k += 4) {
                int jj[4];
                list_quad16(nb, k, base, jj);
                quad(jj);
            }
        } else {
            for (int k = 0; k < nrows; k += 4) {
                int jj[4];
                list_quad32(nb, k, jj);
                quad(jj);
            }
        }
        if (FIXED) {
            range_bad = range_bad || irmax > R.ir2_lim_fx[p];
            const uint64_t mb = (uint64_t)__double_as_longlong(FIX_MAGIC) * (uint64_t)nrows;
            qx -= mb;
            qy -= mb;
            qz -= mb;
        } else {
            const double c = R.c48_h[p];
            fx = fma(c, (double)sx, fx);
            fy = fma(c, (double)sy, fy);
            fz = fma(c, (double)sz, fz);
        }
        if (ENERGY) {
            pe += 0.5 * (4.0 * m.eps[p] * (double)se - (double)cnt * m.vshift[p]);
            vir += 0.5 * 48.0 * m.eps[p] * (double)sv;
            npair += (double)cnt;
        }
        row += base != -1 ? nrows / 2 : nrows;  // 16-bit entries: base >= 0, or a staged window
    }
    if (FIXED) {
        const double inv = 1.0 / FIX_SCALE;
        fx = (double)(int64_t)qx * inv;
        fy = (double)(int64_t)qy * inv;
        fz = (double)(int64_t)qz * inv;
        // the per-pair bound, and a net force beyond which the int64 -> FP64
        // conversion of the sum is no longer exact (2^53 units)
        const double lim = 1.0e8;
        if (range_bad || fabs(fx) > lim || fabs(fy) > lim || fabs(fz) > lim) set_err(d.err, KAMD_DEV_FORCE_RANGE);
    }
    if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) set_err(d.err, KAMD_DEV_NONFINITE);
    if (!KD) {
        d.ax[s] = fx;
        d.ay[s] = fy;
        d.az[s] = fz;
    } else if ((s - S.slot0) < S.n) {
        const double h = 0.5 * dt;
        const double a[3] = {fx, fy, fz};
        const double v[3] = {fma(h, fx, ld_stream(&d.vx[s])), fma(h, fy, ld_stream(&d.vy[s])), fma(h, fz, ld_stream(&d.vz[s]))};
        if (ENERGY) ke2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        drift_core(d, s, R, dt, 0.0, 0.0, h, v, a, mirror_out, d2);
    }
    if (ENERGY) {
        pe = wave_sum(pe);
        vir = wave_sum(vir);
        npair = wave_sum(npair);
        if (KD) ke2 = wave_sum(ke2);
        if (lane_id() == 0) {
            if (KD) d.wred[4 * w + 0] = ke2;
            d.wred[4 * w + 1] = pe;
            d.wred[4 * w + 2] = vir;
            d.wred[4 * w + 3] = npair;
        }
    }
    }
    if (KD) block_disp_max<WPB>(md_out, valid, rep, d2);
}

// The mixed kernel with or without windows (as the lists were built), in
// blocks of WPB wavefronts.
template <bool FIXED, bool ENERGY, bool KD, int WPB>
static void launch_mixed_wpb(const Dev &d, const Model &m, int si, double dt, uint4 *mirror_out, uint32_t *md_out,
                             hipStream_t s)
{
    const int nb = (d.nwaves + WPB - 1) / WPB;
    if (d.stage_ok)
        hipLaunchKernelGGL((k_force_mixed<FIXED, ENERGY, KD, true, WPB>), dim3(nb), dim3(WAVE * WPB), 0, s, d, m, si,
                           dt, mirror_out, md_out);
    else
        hipLaunchKernelGGL((k_force_mixed<FIXED, ENERGY, KD, false, WPB>), dim3(nb), dim3(WAVE * WPB), 0, s, d, m,
                           si, dt, mirror_out, md_out);
}

template <bool FIXED, bool ENERGY, bool KD>
static void launch_mixed(const Dev &d, const Model &m, int si, double dt, uint4 *mirror_out, uint32_t *md_out,
                         int wpb, hipStream_t s)
{
    if (wpb == 1) launch_mixed_wpb<FIXED, ENERGY, KD, 1>(d, m, si, dt, mirror_out, md_out, s);
    else if (wpb == 2) launch_mixed_wpb<FIXED, ENERGY, KD, 2>(d, m, si, dt, mirror_out, md_out, s);
    else launch_mixed_wpb<FIXED, ENERGY, KD, 4>(d, m, si, dt, mirror_out, md_out, s);
}

template <bool ENERGY, bool KD, int WPB>
static void launch_fp64_wpb(const Dev &d, const Model &m, int si, double dt, uint4 *mirror_out, uint32_t *md_out,
                            double4 *pos4_out, hipStream_t s)
{
    const int nb = (d.nwaves + WPB - 1) / WPB;
    hipLaunchKernelGGL((k_force_fp64<ENERGY, KD, WPB>), dim3(nb), dim3(WAVE * WPB), 0, s, d, m, si, dt, mirror_out,
                       md_out, pos4_out);
}

// Force-only launches (md_forces, the last step of a call, Nose-Hoover):
// blocks of WAVES_PER_BLOCK wavefronts.
hipError_t launch_force(const Dev &d, const Model &m, int prec, bool energy, bool step_inc, hipStream_t s)
{
    const int si = step_inc ? 1 : 0;
    constexpr int W4 = WAVES_PER_BLOCK;
    if (prec == 0) {
        hipLaunchKernelGGL(k_pack_pos, dim3((d.npad_total + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, d);
        if (energy)
            launch_fp64_wpb<true, false, W4>(d, m, si, 0.0, nullptr, nullptr, nullptr, s);
        else
            launch_fp64_wpb<false, false, W4>(d, m, si, 0.0, nullptr, nullptr, nullptr, s);
    } else if (prec == 1) {
        if (energy)
            launch_mixed_wpb<false, true, false, W4>(d, m, si, 0.0, nullptr, nullptr, s);
        else
            launch_mixed_wpb<false, false, false, W4>(d, m, si, 0.0, nullptr, nullptr, s);
    } else {
        if (energy)
            launch_mixed_wpb<true, true, false, W4>(d, m, si, 0.0, nullptr, nullptr, s);
        else
            launch_mixed_wpb<true, false, false, W4>(d, m, si, 0.0, nullptr, nullptr, s);
    }
    return hipGetLastError();
}

hipError_t launch_pack_pos(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_pos, dim3((d.npad_total + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_force_kd(const Dev &d, const Model &m, int prec, double dt, uint4 *mirror_out, uint32_t *md_out,
                           double4 *pos4_out, bool energy, int wpb, hipStream_t s)
{
    if (wpb != 1 && wpb != 2 && wpb != 4) return hipErrorInvalidValue;
    if (prec == 0) {
        if (!d.pos4 || !pos4_out || pos4_out == d.pos4) return hipErrorInvalidValue;
        if (energy) {
            if (wpb == 1) launch_fp64_wpb<true, true, 1>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
            else if (wpb == 2) launch_fp64_wpb<true, true, 2>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
            else launch_fp64_wpb<true, true, 4>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
        } else {
            if (wpb == 1) launch_fp64_wpb<false, true, 1>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
            else if (wpb == 2) launch_fp64_wpb<false, true, 2>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
            else launch_fp64_wpb<false, true, 4>(d, m, 1, dt, mirror_out, md_out, pos4_out, s);
        }
    } else if (prec == 1) {
        if (energy)
            launch_mixed<false, true, true>(d, m, 1, dt, mirror_out, md_out, wpb, s);
        else
            launch_mixed<false, false, true>(d, m, 1, dt, mirror_out, md_out, wpb, s);
    } else if (prec == 2) {
        if (energy)
            launch_mixed<true, true, true>(d, m, 1, dt, mirror_out, md_out, wpb, s);
        else
            launch_mixed<true, false, true>(d, m, 1, dt, mirror_out, md_out, wpb, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kamd
