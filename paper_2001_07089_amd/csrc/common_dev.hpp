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

__device__ inline int wave_id_remapped()
{
    int b = xcd_block(blockIdx.x, gridDim.x);
    return b * WAVES_PER_BLOCK + (threadIdx.x >> 6);
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

// Rebuild decision of replica r for the running step.  Every kernel of the
// rebuild chain evaluates it identically: nothing it reads changes before the
// force kernel of the same step closes the check.
__device__ inline bool rebuild_flag(const Dev &d, int r)
{
    return d.rb_force[r] != 0 || (double)__uint_as_float(d.maxdisp[r]) > d.rep[r].disp_thr2;
}

}  // namespace kamd
