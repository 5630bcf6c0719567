// common_dev.hpp -- small device helpers of the HIP kernels.
#pragma once
#include "kamd_internal.hpp"

namespace kamd {

// Wavefront index of this thread for kernels launched with BLOCK threads over
// the slot range, with blocks remapped so that each of the 8 XCDs (one L2
// each) receives a contiguous range of slots: hardware dispatches block b to
// XCD b % 8.
__device__ inline int xcd_block(int b, int nb)
{
    int q = nb >> 3, r = nb & 7;
    int x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <int WPB = WAVES_PER_BLOCK>
__device__ inline int wave_id_remapped()
{
    int b = xcd_block(blockIdx.x, gridDim.x);
    return b * WPB + (threadIdx.x >> 6);
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Wavefront reductions (all 64 lanes must be active).
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// u32 fixed-point coordinate of u in [0, L): round(u * 2^32 / L) mod 2^32.
__device__ inline uint32_t to_fix(double u, double invL)
{
    double q = rint(u * invL * 4294967296.0);
    if (q >= 4294967296.0) q -= 4294967296.0;
    if (q < 0.0) q += 4294967296.0;
    return (uint32_t)q;
}

// Cell coordinate of a fixed-point coordinate on an nc grid: floor(u * nc / 2^32).
__device__ inline int fix_cell(uint32_t u, int nc) { return (int)__umulhi(u, (uint32_t)nc); }

__device__ inline void set_err(uint32_t *err, uint32_t bit) { atomicOr(err, bit); }

// Streaming accesses: data that a step reads or writes once (the particle's
// own state, the 32-bit list parts), loaded and stored non-temporally so that
// it does not displace the neighbour positions the gathers of the force
// kernels keep reusing from the caches.  (Measured at N = 2^20: the fused
// step kernel 0.227 -> 0.209 ms.  The 16-bit list parts are not marked: each
// of their words is read twice, by consecutive passes.)
template <typename T>
__device__ inline T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ inline void st_stream(T v, T *p)
{
    __builtin_nontemporal_store(v, p);
}
__device__ inline uint4 ld_stream(const uint4 *p)
{
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ inline int4 ld_stream(const int4 *p)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}

// ------------------------------------------------ integration helpers
__device__ inline double wrap_img(double u, double L, double invL, int32_t &img)
{
    double k = floor(u * invL);
    u = fma(-k, L, u);
    if (u >= L) { u -= L; k += 1.0; }
    if (u < 0.0) { u += L; k -= 1.0; }
    img += (int32_t)k;
    return u;
}

// Position half of a velocity-Verlet step for slot s, from the velocity v at
// the start of the step and the acceleration a: v_h = v + c (a - (xi + xi_a)
// v), r += dt (v + dt/2 (a - xi v)), wrap into [0, L) counting images.
// Stores r, v_h and the image counters, writes the new u32 mirror into
// mirror_out and returns the squared displacement since the last list build
// in d2.  NVE: xi = xi_a = 0, c = dt/2.
__device__ inline void drift_core(const Dev &d, int s, const RepInfo &R, double dt, double xi, double xia,
                                  double c, const double v[3], const double a[3], uint4 *mirror_out, float &d2)
{
    const int np = d.npad_total;
    const double L = R.L, invL = R.invL;
    double r[3] = {ld_stream(&d.x[s]), ld_stream(&d.y[s]), ld_stream(&d.z[s])};
    double vn[3];
    int32_t im[3] = {ld_stream(&d.img[s]), ld_stream(&d.img[np + s]), ld_stream(&d.img[2 * np + s])};
    uint32_t q[3];
    bool fin = true;
    double step2 = 0.0;  // squared length of this step's move (runaway check)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double g = a[k] - xi * v[k];
        const double u = fma(0.5 * dt, g, v[k]);
        step2 = fma(u, u, step2);
        r[k] = fma(dt, u, r[k]);
        vn[k] = fma(c, a[k] - (xi + xia) * v[k], v[k]);
        fin = fin && isfinite(r[k]) && isfinite(vn[k]);
        r[k] = wrap_img(r[k], L, invL, im[k]);
        q[k] = to_fix(r[k], invL);
    }
    st_stream(r[0], &d.x[s]); st_stream(r[1], &d.y[s]); st_stream(r[2], &d.z[s]);
    st_stream(vn[0], &d.vx[s]); st_stream(vn[1], &d.vy[s]); st_stream(vn[2], &d.vz[s]);
    st_stream(im[0], &d.img[s]); st_stream(im[1], &d.img[np + s]); st_stream(im[2], &d.img[2 * np + s]);
    mirror_out[s] = make_uint4(q[0], q[1], q[2], 0u);  // gathered by the next step: cached
    const uint4 b = ld_stream(&d.mbuild[s]);
    const float ex = (float)(int)(q[0] - b.x), ey = (float)(int)(q[1] - b.y),
                ez = (float)(int)(q[2] - b.z);
    const float h = (float)(R.L * 2.3283064365386963e-10);
    d2 = (ex * ex + ey * ey + ez * ez) * (h * h);
    if (!fin) set_err(d.err, KAMD_DEV_NONFINITE);
    if (step2 * (dt * dt) > R.run2) set_err(d.err, KAMD_DEV_RUNAWAY);
}

__device__ inline void drift_one(const Dev &d, int s, int rep, double dt, double xi, double xia,
                                 double c, uint4 *mirror_out, float &d2)
{
    const double v[3] = {d.vx[s], d.vy[s], d.vz[s]};
    const double a[3] = {d.ax[s], d.ay[s], d.az[s]};
    drift_core(d, s, d.rep[rep], dt, xi, xia, c, v, a, mirror_out, d2);
}

// Per-replica maximum of the wavefront maxima of one block, one atomicMax per
// replica present in the block (a block holds WPB consecutive wavefronts,
// which may straddle two replicas).  All threads of the block must call it.
template <int WPB = WAVES_PER_BLOCK>
__device__ inline void block_disp_max(uint32_t *maxdisp, bool valid, int rep, float d2)
{
    __shared__ float wmax[WPB];
    __shared__ int wrep[WPB];
    d2 = wave_max(d2);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        wmax[wv] = d2;
        wrep[wv] = valid ? rep : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // read first: the maximum only grows during the step, so most blocks
        // find it already larger and skip the atomic
        auto push = [&](int r, float m) {
            const uint32_t bits = __float_as_uint(m);
            const uint32_t cur = __hip_atomic_load(&maxdisp[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (bits > cur) atomicMax(&maxdisp[r], bits);
        };
        int r = -1;
        float m = 0.0f;
        for (int k = 0; k < WPB; ++k) {
            if (wrep[k] != r) {
                if (r >= 0) push(r, m);
                r = wrep[k];
                m = 0.0f;
            }
            m = fmaxf(m, wmax[k]);
        }
        if (r >= 0) push(r, m);
    }
}

}  // namespace kamd
