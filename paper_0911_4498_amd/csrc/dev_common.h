// dev_common.h -- device helpers shared by the kernels of the single-series path:
// four-step twiddles, wave sums, the counter-based normal generator, the XCD-aware
// block order and FP64 dot products of FP32 rows.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ssa_internal.h"

namespace ssa {

__device__ __forceinline__ float2 twiddle_mp(const ConvGeom& g, long long t) {
    const long long mask = (1LL << g.tw_shift) - 1;
    return cmul(g.tw_hi[t >> g.tw_shift], g.tw_lo[t & mask]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the workgroup (every thread gets it; a fixed order: waves, then wave 0, 1, ...).
// sh holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    __syncthreads();
    return s;
}

// sum_c hs[c]^2 over ncols values in LDS, formed by every wave on its own (lane l adds
// c = l, l + 64, ... in order, then an xor butterfly): every lane of every wave gets the
// same bits (each butterfly stage adds the same two values, in either order), with no
// barrier.
__device__ __forceinline__ double sumsq_allwave(const double* hs, int ncols) {
    const int lane = threadIdx.x & 63;
    double v = 0.0;
    for (int c = lane; c < ncols; c += 64) v += hs[c] * hs[c];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3").
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
        const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Standard normal number for element t of stream `ctr` (Box-Muller on two uniforms).
__device__ __forceinline__ float gauss(unsigned long long seed, unsigned long long ctr, long long t) {
    uint32_t c[4] = {(uint32_t)t, (uint32_t)((unsigned long long)t >> 32), (uint32_t)ctr,
                     (uint32_t)(ctr >> 32)};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967296.0);  // (0, 1]
    const double u2 = (double)c[1] * (1.0 / 4294967296.0);
    return (float)(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup i to XCD i mod 8), and each
// XCD has its own L2.  Column blocks of passes 1 and 3 read and write runs of CB
// complex values, so neighbouring blocks share 128-byte lines: give each XCD a
// contiguous run of blocks so that those neighbours meet in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    if (nb % kXcds != 0) return b;
    return (b % kXcds) * (nb / kXcds) + b / kXcds;
}

// 4 consecutive rows t..t+3 (t a multiple of 4, t < n) of a column whose
// allocation is padded to a multiple of 64 floats; rows >= n read as zero.
__device__ __forceinline__ float4 rows4(const float* __restrict__ col, long long t, long long n) {
    float4 v = *reinterpret_cast<const float4*>(col + t);
    if (t + 3 >= n) {
        if (t + 1 >= n) v.y = 0.0f;
        if (t + 2 >= n) v.z = 0.0f;
        if (t + 3 >= n) v.w = 0.0f;
    }
    return v;
}

__device__ __forceinline__ double dot4(float4 a, float4 b) {
    return (double)a.x * (double)b.x + (double)a.y * (double)b.y + (double)a.z * (double)b.z +
           (double)a.w * (double)b.w;
}

}  // namespace ssa
