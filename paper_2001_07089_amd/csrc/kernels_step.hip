// kernels_step.hip -- integration, thermostats, reductions and the transfers
// between the caller's particle order and the internal slot order.
//
// Velocity Verlet (Sec. II.D, Eqs. (velVerletPos),(velVerletVel); the order of
// the time loop in Sec. III.E) is split around the force evaluation:
//   drift:  v_h = v + c (a - (xi + xi_a) v);  r += dt (v + dt/2 (a - xi v));
//           wrap into [0, L) counting images; refresh the u32 mirror and the
//           displacement since the last list build
//   force:  a = F(r)
//   kick:   v = v_h + c a
// With xi = xi_a = 0 and c = dt/2 this is the NVE step exactly
// (r += v dt + a dt^2/2, v += a dt/2 twice).  With the Nose-Hoover values of
// Appendix B (c = dt/2 (1 - dt/2 xi_a)) the two velocity halves add up to
// Eq. (ridotKVLRoman) and the position update is Eq. (Noseupdate_ri).
//
// All state is FP64 in every precision mode.  Per-wavefront partial sums are
// written to wred and reduced per replica in a fixed order (deterministic).
#include "common_dev.hpp"

#include <algorithm>

namespace kamd {

struct SlotCtx {
    int w, s;
    bool real;
    int rep;
};

__device__ inline bool slot_ctx(const Dev &d, SlotCtx &c)
{
    c.w = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    c.s = 0;
    c.real = false;
    c.rep = -1;
    if (c.w >= d.nwaves) return false;
    const SegInfo &S = d.seg[d.wave_seg[c.w]];
    c.s = c.w * WAVE + lane_id();
    c.real = (c.s - S.slot0) < S.n;
    c.rep = S.rep;
    return true;
}

__global__ __launch_bounds__(BLOCK) void k_drift(Dev d, double dt, int nh)
{
    SlotCtx c;
    const bool valid = slot_ctx(d, c);
    float d2 = 0.0f;
    if (valid && c.real) {
        double xi = 0.0, xia = 0.0, ck = 0.5 * dt;
        if (nh) {
            const RepDyn &D = d.dyn[c.rep];
            xi = D.xi; xia = D.xia; ck = D.c_kick;
        }
        drift_one(d, c.s, c.rep, dt, xi, xia, ck, d.mirror, d2);
    }
    block_disp_max(d.maxdisp, valid, valid ? c.rep : -1, d2);
}

// v = v_h + c a, with c the replica's kick factor; optional per-wave sum v^2.
__global__ __launch_bounds__(BLOCK) void k_kick(Dev d, double c_nve, int nh, int want_ke)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    double k2 = 0.0;
    if (c.real) {
        const double ck = nh ? d.dyn[c.rep].c_kick : c_nve;
        const int s = c.s;
        const double vx = fma(ck, d.ax[s], d.vx[s]);
        const double vy = fma(ck, d.ay[s], d.vy[s]);
        const double vz = fma(ck, d.az[s], d.vz[s]);
        d.vx[s] = vx; d.vy[s] = vy; d.vz[s] = vz;
        k2 = vx * vx + vy * vy + vz * vz;
    }
    if (want_ke) {
        k2 = wave_sum(k2);
        if (lane_id() == 0) d.wred[4 * c.w + 0] = k2;
    }
}

// NVE only: the closing half-kick of one step fused with the drift of the
// next (both use the same acceleration), one pass over the state.
__global__ __launch_bounds__(BLOCK) void k_kick_drift(Dev d, double dt, int want_ke)
{
    SlotCtx c;
    const bool valid = slot_ctx(d, c);
    float d2 = 0.0f;
    double k2 = 0.0;
    if (valid && c.real) {
        const int s = c.s;
        const double h = 0.5 * dt;
        const double vx = fma(h, d.ax[s], d.vx[s]);
        const double vy = fma(h, d.ay[s], d.vy[s]);
        const double vz = fma(h, d.az[s], d.vz[s]);
        k2 = vx * vx + vy * vy + vz * vz;
        d.vx[s] = vx; d.vy[s] = vy; d.vz[s] = vz;
        drift_one(d, s, c.rep, dt, 0.0, 0.0, h, d.mirror, d2);
    }
    if (want_ke && valid) {
        k2 = wave_sum(k2);
        if (lane_id() == 0) d.wred[4 * c.w + 0] = k2;
    }
    block_disp_max(d.maxdisp, valid, valid ? c.rep : -1, d2);
}

// Per-replica sum of the 4 per-wave partials (fixed order).  what: 0 -> rsum.
// Each thread reads a wave's four partials as one 32-byte load, four waves
// (BLOCK apart) per pass, so that a replica of many waves (16,384 at N =
// 2^20) is read in a quarter of the dependent passes.
__global__ __launch_bounds__(BLOCK) void k_rep_reduce(Dev d, int mask)
{
    __shared__ double red[4][BLOCK];
    const int r = blockIdx.x;
    const RepInfo &R = d.rep[r];
    const double4 *wr = reinterpret_cast<const double4 *>(d.wred);
    auto pick = [mask](const double4 &v, int k) __attribute__((always_inline)) {
        const double x = k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
        return (mask & (1 << k)) ? x : 0.0;
    };
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int w = R.wave0 + threadIdx.x;
    for (; w + 3 * BLOCK < R.wave1; w += 4 * BLOCK) {
        const double4 v0 = wr[w], v1 = wr[w + BLOCK], v2 = wr[w + 2 * BLOCK], v3 = wr[w + 3 * BLOCK];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] += (pick(v0, k) + pick(v1, k)) + (pick(v2, k) + pick(v3, k));
    }
    for (; w < R.wave1; w += BLOCK) {
        const double4 v = wr[w];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] += pick(v, k);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 4 && (mask & (1 << threadIdx.x))) d.rsum[4 * r + threadIdx.x] = red[threadIdx.x][0];
}

// Nose-Hoover scalars before the drift (Appendix B): with K = sum v(t)^2,
// G = (K - d N T) / Q: ln s += xi dt + G dt^2/2 (Eq. (Noseupdate_lns)),
// xi_a = xi + G dt (Eq. (Noseupdate_xiapprox)), c = dt/2 (1 - dt/2 xi_a).
__global__ void k_nh_begin(Dev d, double dt, const double *Q)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    const RepInfo &R = d.rep[r];
    RepDyn &D = d.dyn[r];
    const double X = (double)d.dim * (double)R.n;  // degrees of freedom d N
    const double G = (D.K2 - X * R.T) / Q[r];
    D.lns += D.xi * dt + 0.5 * G * dt * dt;
    D.xia = D.xi + G * dt;
    D.c_kick = 0.5 * dt * (1.0 - 0.5 * dt * D.xia);
}

// After the closing kick: xi(t+dt) = xi + dt/2 (G + G'), G' from the new
// velocities (Eq. (FoxAndersen_ydottplush) for y = ln s); K <- sum v(t+dt)^2.
__global__ void k_nh_end(Dev d, double dt, const double *Q)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    const RepInfo &R = d.rep[r];
    RepDyn &D = d.dyn[r];
    const double X = (double)d.dim * (double)R.n;  // degrees of freedom d N
    const double K1 = d.rsum[4 * r + 0];
    const double G = (D.K2 - X * R.T) / Q[r];
    const double G1 = (K1 - X * R.T) / Q[r];
    D.xi = D.xi + 0.5 * dt * (G + G1);
    D.K2 = K1;
}

// K <- rsum[0] (after a sum-v^2 reduction).
__global__ void k_set_k2(Dev d)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    d.dyn[r].K2 = d.rsum[4 * r + 0];
}

__global__ __launch_bounds__(BLOCK) void k_ke_partial(Dev d)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    double k2 = 0.0;
    if (c.real) {
        const int s = c.s;
        k2 = d.vx[s] * d.vx[s] + d.vy[s] * d.vy[s] + d.vz[s] * d.vz[s];
    }
    k2 = wave_sum(k2);
    if (lane_id() == 0) d.wred[4 * c.w + 0] = k2;
}

// ------------------------------------------------------------ Philox + MB
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// products and xors, Weyl key increments between rounds.
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// (2k+1)/2^53 with k the 26 high bits of a followed by the 26 high bits of b.
__device__ inline double uni_open(uint32_t a, uint32_t b)
{
    const uint64_t k = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
    return (double)(2 * k + 1) * 0x1p-53;
}

// Three standard normals for (seed, replica, draw tag, particle id) by the
// Box-Muller transform; counter {id, tag, replica, block}.
__device__ inline void gauss3(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t id, double g[3])
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const double twopi = 6.283185307179586476925286766559;
    uint32_t c[4] = {id, tag, rep, 0u};
    philox10(c, k0, k1);
    double u1 = uni_open(c[0], c[1]), u2 = uni_open(c[2], c[3]);
    double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(twopi * u2, &sn, &cs);
    g[0] = rad * cs;
    g[1] = rad * sn;
    uint32_t e[4] = {id, tag, rep, 1u};
    philox10(e, k0, k1);
    u1 = uni_open(e[0], e[1]);
    u2 = uni_open(e[2], e[3]);
    rad = sqrt(-2.0 * log(u1));
    g[2] = rad * cos(twopi * u2);
}

// Maxwell-Boltzmann flow chart (Sec. II.E.1), step 1 (step 2 is void for
// unit masses): Gaussian velocities of standard deviation sqrt(T); per-wave
// sums of the components for step 3.
__global__ __launch_bounds__(BLOCK) void k_mb_draw(Dev d, uint32_t tag, int tag_from_device)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    if (tag_from_device) tag = (uint32_t)d.counters[1];
    double sv[3] = {0.0, 0.0, 0.0};
    if (c.real) {
        const RepInfo &R = d.rep[c.rep];
        const uint32_t local = (uint32_t)((int64_t)d.id[c.s] - R.caller_off);
        double g[3];
        gauss3(R.seed, (uint32_t)c.rep, tag, local, g);
        const double sg = sqrt(R.T);
        sv[0] = sg * g[0]; sv[1] = sg * g[1]; sv[2] = d.dim == 2 ? 0.0 : sg * g[2];
        d.vx[c.s] = sv[0]; d.vy[c.s] = sv[1]; d.vz[c.s] = sv[2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) sv[k] = wave_sum(sv[k]);
    if (lane_id() == 0) {
        d.wred[4 * c.w + 0] = sv[0];
        d.wred[4 * c.w + 1] = sv[1];
        d.wred[4 * c.w + 2] = sv[2];
        d.wred[4 * c.w + 3] = 0.0;
    }
}

// Step 3: subtract the centre-of-mass velocity; per-wave sum v^2 for step 4.
__global__ __launch_bounds__(BLOCK) void k_mb_center(Dev d)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    double k2 = 0.0;
    if (c.real) {
        const double inv = 1.0 / (double)d.rep[c.rep].n;
        const double *m = d.rsum + 4 * c.rep;
        const double vx = d.vx[c.s] - m[0] * inv;
        const double vy = d.vy[c.s] - m[1] * inv;
        const double vz = d.vz[c.s] - m[2] * inv;
        d.vx[c.s] = vx; d.vy[c.s] = vy; d.vz[c.s] = vz;
        k2 = vx * vx + vy * vy + vz * vz;
    }
    k2 = wave_sum(k2);
    if (lane_id() == 0) d.wred[4 * c.w + 0] = k2;
}

// Step 4: rescale so that sum v^2 = 3 N T (Eq. (equip3N)).  A replica of one
// particle has no velocity left after step 3 and stays at rest.
__global__ __launch_bounds__(BLOCK) void k_mb_scale(Dev d)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    if (!c.real) return;
    const RepInfo &R = d.rep[c.rep];
    const double s2 = d.rsum[4 * c.rep + 0];
    const double f = s2 > 0.0 ? sqrt((double)d.dim * R.T * (double)R.n / s2) : 0.0;
    d.vx[c.s] *= f;
    d.vy[c.s] *= f;
    d.vz[c.s] *= f;
}

// Velocities of every particle of replica r times f[r] (f: device, [nrep]).
__global__ __launch_bounds__(BLOCK) void k_scale_v(Dev d, const double *f)
{
    SlotCtx c;
    if (!slot_ctx(d, c) || !c.real) return;
    const double a = f[c.rep];
    d.vx[c.s] *= a;
    d.vy[c.s] *= a;
    d.vz[c.s] *= a;
}

// ------------------------------------------------------------- transfers
struct Arr9 {
    const double *p[9];
};

__global__ __launch_bounds__(BLOCK) void k_import(Dev d, Arr9 a, const int32_t *img)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    if (!c.real) return;
    const int s = c.s;
    const int np = d.npad_total;
    const int g = d.id[s];
    const RepInfo &R = d.rep[c.rep];
    double *dst[9] = {d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az};
    int32_t im[3] = {0, 0, 0};
    if (img) { im[0] = img[g]; im[1] = img[d.n_total + g]; im[2] = img[2 * d.n_total + g]; }
    for (int k = 0; k < 9; ++k)
        if (a.p[k]) {
            double v = a.p[k][g];
            if (k < 3) v = wrap_img(v, R.L, R.invL, im[k]);
            dst[k][s] = v;
        }
    if (d.dim == 2) {  // planar: z, vz and az are zero by definition
        d.z[s] = 0.0;
        d.vz[s] = 0.0;
        d.az[s] = 0.0;
        im[2] = 0;
    }
    d.img[s] = im[0]; d.img[np + s] = im[1]; d.img[2 * np + s] = im[2];
    d.mirror[s] = make_uint4(to_fix(d.x[s], R.invL), to_fix(d.y[s], R.invL), to_fix(d.z[s], R.invL), 0u);
}

struct Arr9w {
    double *p[9];
};

__global__ __launch_bounds__(BLOCK) void k_export(Dev d, Arr9w a, int32_t *img)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    if (!c.real) return;
    const int s = c.s;
    const int np = d.npad_total;
    const int g = d.id[s];
    const double *src[9] = {d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az};
    for (int k = 0; k < 9; ++k)
        if (a.p[k]) a.p[k][g] = src[k][s];
    if (img) {
        img[g] = d.img[s];
        img[d.n_total + g] = d.img[np + s];
        img[2 * d.n_total + g] = d.img[2 * np + s];
    }
}

__global__ __launch_bounds__(BLOCK) void k_mirror(Dev d)
{
    SlotCtx c;
    if (!slot_ctx(d, c)) return;
    if (!c.real) return;
    const double invL = d.rep[c.rep].invL;
    d.mirror[c.s] = make_uint4(to_fix(d.x[c.s], invL), to_fix(d.y[c.s], invL), to_fix(d.z[c.s], invL), 0u);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_zero_f64(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Copy rsum[r][0..3] into out[r][0..3] (observable staging).
__global__ void k_store_obs(Dev d, double *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    for (int k = 0; k < 4; ++k) out[4 * r + k] = d.rsum[4 * r + k];
}

// (PE, W) of each replica from rsum[1..2] into out[r][0..1].
__global__ void k_store_pe_w(Dev d, double *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.nrep) return;
    out[2 * r + 0] = d.rsum[4 * r + 1];
    out[2 * r + 1] = d.rsum[4 * r + 2];
}

// One row of the observables ring per replica, from the per-replica sums in
// rsum (Eq. (EsysNpart): E_tot = KE + PE; Eq. (equip3N): T = 2 KE / (d N)).
// A row may be filled in two launches (PE and W before a velocity redraw, KE
// after it); mask 4 completes it and advances the row counter.  One block.
__global__ __launch_bounds__(BLOCK) void k_sample(Dev d, int mask)
{
    const int idx = d.counters[2];
    const int slot = idx % d.ring_cap;
    for (int r = threadIdx.x; r < d.nrep; r += BLOCK) {
        double *row = d.ring + ((size_t)r * d.ring_cap + slot) * 6;
        const double *rs = d.rsum + 4 * r;
        if (mask & 1) row[1] = 0.5 * rs[0];
        if (mask & 2) {
            row[2] = rs[1];
            row[5] = rs[2];
        }
        if (mask & 4) {
            row[0] = (double)d.counters[1];
            row[3] = row[1] + row[2];
            row[4] = 2.0 * row[1] / ((double)d.dim * (double)d.rep[r].n);
        }
    }
    __syncthreads();
    if ((mask & 4) && threadIdx.x == 0) d.counters[2] = idx + 1;
}

// ------------------------------------------------------------- launchers
static inline int nblk(const Dev &d) { return (d.nwaves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK; }

hipError_t launch_drift(const Dev &d, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_drift, dim3(nblk(d)), dim3(BLOCK), 0, s, d, dt, 0);
    return hipGetLastError();
}
hipError_t launch_drift_nh(const Dev &d, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_drift, dim3(nblk(d)), dim3(BLOCK), 0, s, d, dt, 1);
    return hipGetLastError();
}
hipError_t launch_kick_nve(const Dev &d, double dt, bool want_ke, hipStream_t s)
{
    hipLaunchKernelGGL(k_kick, dim3(nblk(d)), dim3(BLOCK), 0, s, d, 0.5 * dt, 0, want_ke ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_kick_nh(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_kick, dim3(nblk(d)), dim3(BLOCK), 0, s, d, 0.0, 1, 1);
    return hipGetLastError();
}
hipError_t launch_kick_drift(const Dev &d, double dt, bool want_ke, hipStream_t s)
{
    hipLaunchKernelGGL(k_kick_drift, dim3(nblk(d)), dim3(BLOCK), 0, s, d, dt, want_ke ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_rep_reduce(const Dev &d, int mask, hipStream_t s)
{
    hipLaunchKernelGGL(k_rep_reduce, dim3(d.nrep), dim3(BLOCK), 0, s, d, mask);
    return hipGetLastError();
}
hipError_t launch_nh_begin(const Dev &d, double dt, const double *Q, hipStream_t s)
{
    hipLaunchKernelGGL(k_nh_begin, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, dt, Q);
    return hipGetLastError();
}
hipError_t launch_nh_end(const Dev &d, double dt, const double *Q, hipStream_t s)
{
    hipLaunchKernelGGL(k_nh_end, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, dt, Q);
    return hipGetLastError();
}
hipError_t launch_set_k2(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_k2, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_ke_partial(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_ke_partial, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_mb_draw(const Dev &d, uint32_t tag, hipStream_t s)
{
    hipLaunchKernelGGL(k_mb_draw, dim3(nblk(d)), dim3(BLOCK), 0, s, d, tag, 0);
    return hipGetLastError();
}
hipError_t launch_mb_draw_dev(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_mb_draw, dim3(nblk(d)), dim3(BLOCK), 0, s, d, 0u, 1);
    return hipGetLastError();
}
hipError_t launch_mb_center(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_mb_center, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_mb_scale(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_mb_scale, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_scale_v(const Dev &d, const double *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_v, dim3(nblk(d)), dim3(BLOCK), 0, s, d, f);
    return hipGetLastError();
}
hipError_t launch_import(const Dev &d, const double *const *arr, const int32_t *img, hipStream_t s)
{
    Arr9 a;
    for (int k = 0; k < 9; ++k) a.p[k] = arr[k];
    hipLaunchKernelGGL(k_import, dim3(nblk(d)), dim3(BLOCK), 0, s, d, a, img);
    return hipGetLastError();
}
hipError_t launch_export(const Dev &d, double *const *arr, int32_t *img, hipStream_t s)
{
    Arr9w a;
    for (int k = 0; k < 9; ++k) a.p[k] = arr[k];
    hipLaunchKernelGGL(k_export, dim3(nblk(d)), dim3(BLOCK), 0, s, d, a, img);
    return hipGetLastError();
}
hipError_t launch_mirror(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_mirror, dim3(nblk(d)), dim3(BLOCK), 0, s, d);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s) { return launch_fill_i32(p, n, 0, s); }
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_f64, dim3(nb), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_store_pe_w(const Dev &d, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_store_pe_w, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, out);
    return hipGetLastError();
}
hipError_t launch_sample(const Dev &d, int mask, hipStream_t s)
{
    if (!d.ring || d.ring_cap <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample, dim3(1), dim3(BLOCK), 0, s, d, mask);
    return hipGetLastError();
}
hipError_t launch_store_obs(const Dev &d, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_store_obs, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, out);
    return hipGetLastError();
}

}  // namespace kamd
