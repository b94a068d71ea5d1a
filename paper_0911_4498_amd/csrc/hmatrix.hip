// hmatrix.hip -- kernels of structural-change detection (the H-matrix of
// heterogeneity indices, eq. g): base-window copies, the squared projections
// of every lagged vector on each base window's eigenvectors, the lagged-vector
// energies, and the window sums that give each index.
//
// With u_t (t in I) the eigenvectors of base window i, lagged vector p of the
// series X_p = f[p .. p+L), and test window j made of X_j .. X_{j+K2-1}:
//   num_ij = sum_{m<K2} sum_t (u_t . X_{j+m})^2,  den_j = sum_{m<K2} |X_{j+m}|^2,
//   g_ij = (den_j - num_ij) / den_j,
// which is the distance form of eq. g because the u_t are orthonormal.  The
// window sums come from prefix sums along p (FP64).
#include <hip/hip_runtime.h>

#include "ssa_hmatrix.h"

namespace ssa {
namespace hm {

constexpr int kTile = 256;  // lagged vectors per workgroup in k_corr

// out[i*B + t] = f[i + t]: the base windows as separate series
__global__ __launch_bounds__(256) void k_windows(const double* __restrict__ f, long long B, long long MB,
                                                 double* __restrict__ out) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= MB * B) return;
    const long long i = idx / B, t = idx - i * B;
    out[idx] = f[i + t];
}

// c2[i*P + p] = sum_{t in I} (u_t^(i) . X_p)^2 for p < P = N - L + 1, FP64 sums of
// exact FP32 products.  Grid (ceil(P / kTile), MB); LDS: the nI vectors of base
// window i and the kTile + L - 1 series values the tile's lagged vectors cover.
__global__ __launch_bounds__(kTile) void k_corr(const double* __restrict__ f, long long N, long long L,
                                                const float* __restrict__ U, int k, const int* __restrict__ I,
                                                int nI, double* __restrict__ c2) {
    extern __shared__ float smem[];
    float* u = smem;                 // nI x L
    float* x = smem + (long long)nI * L;  // kTile + L - 1
    const long long P = N - L + 1;
    const long long i = blockIdx.y;
    const long long p0 = (long long)blockIdx.x * kTile;
    const float* Ui = U + i * L * k;  // u_t at Ui + t*L
    for (long long idx = threadIdx.x; idx < (long long)nI * L; idx += kTile) {
        const int q = (int)(idx / L);
        const long long l = idx - (long long)q * L;
        u[idx] = Ui[(long long)(I[q] - 1) * L + l];
    }
    for (long long idx = threadIdx.x; idx < kTile + L - 1; idx += kTile) {
        const long long m = p0 + idx;
        x[idx] = m < N ? (float)f[m] : 0.0f;
    }
    __syncthreads();
    const long long p = p0 + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int q = 0; q < nI; ++q) {
        const float* uq = u + (long long)q * L;
        double acc = 0.0;
        for (long long l = 0; l < L; ++l) acc += (double)uq[l] * (double)x[threadIdx.x + l];
        s += acc * acc;
    }
    c2[i * P + p] = s;
}

// sq[p] = |X_p|^2 (FP64 sums of exact FP32 squares), p < P
__global__ __launch_bounds__(256) void k_energy(const double* __restrict__ f, long long N, long long L,
                                                double* __restrict__ sq) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= N - L + 1) return;
    double s = 0.0;
    for (long long l = 0; l < L; ++l) {
        const double v = (double)(float)f[p + l];
        s += v * v;
    }
    sq[p] = s;
}

// In-place inclusive prefix sums of each row of a (rows x P) FP64 array, one
// workgroup per row, 256-value chunks in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_scan_rows(double* __restrict__ a, long long P) {
    __shared__ double wtot[4];
    double* row = a + (long long)blockIdx.x * P;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double carry = 0.0;
    for (long long c0 = 0; c0 < P; c0 += 256) {
        const long long p = c0 + tid;
        double v = p < P ? row[p] : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double y = __shfl_up(v, off, 64);
            if (lane >= off) v += y;
        }
        if (lane == 63) wtot[wave] = v;
        __syncthreads();
        double before = carry;
        for (int w = 0; w < wave; ++w) before += wtot[w];
        const double total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
        if (p < P) row[p] = before + v;
        __syncthreads();
        carry += total;
    }
}

// G[i*MT + j] = (den_j - num_ij) / den_j from the prefix sums S (rows of squared
// projections) and Q (lagged-vector energies); 0 for a test window without energy.
__global__ __launch_bounds__(256) void k_rows(const double* __restrict__ S, const double* __restrict__ Q,
                                              long long P, long long MT, long long K2, double* __restrict__ G) {
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long i = blockIdx.y;
    if (j >= MT) return;
    const double* row = S + i * P;
    const double num = row[j + K2 - 1] - (j > 0 ? row[j - 1] : 0.0);
    const double den = Q[j + K2 - 1] - (j > 0 ? Q[j - 1] : 0.0);
    G[i * MT + j] = den > 0.0 ? fmax(den - num, 0.0) / den : 0.0;
}

}  // namespace hm

hipError_t launch_hm_windows(const double* f, long long B, long long MB, double* out, hipStream_t s) {
    const long long n = MB * B;
    hipLaunchKernelGGL(hm::k_windows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, B, MB, out);
    return hipGetLastError();
}

hipError_t launch_hm_corr(const double* f, long long N, long long L, const float* U, int k, const int* I, int nI,
                          long long MB, double* c2, hipStream_t s) {
    const long long P = N - L + 1;
    const size_t lds = sizeof(float) * ((size_t)nI * L + hm::kTile + L - 1);
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hm::k_corr),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(hm::k_corr, dim3((unsigned)((P + hm::kTile - 1) / hm::kTile), (unsigned)MB),
                       dim3(hm::kTile), lds, s, f, N, L, U, k, I, nI, c2);
    return hipGetLastError();
}

hipError_t launch_hm_energy(const double* f, long long N, long long L, double* sq, hipStream_t s) {
    const long long P = N - L + 1;
    hipLaunchKernelGGL(hm::k_energy, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, f, N, L, sq);
    return hipGetLastError();
}

hipError_t launch_hm_rows(double* c2, double* sq, long long P, long long MB, long long MT, long long K2,
                          double* G, hipStream_t s) {
    hipLaunchKernelGGL(hm::k_scan_rows, dim3((unsigned)MB), dim3(256), 0, s, c2, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hm::k_scan_rows, dim3(1), dim3(256), 0, s, sq, P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hm::k_rows, dim3((unsigned)((MT + 255) / 256), (unsigned)MB), dim3(256), 0, s, c2, sq, P,
                       MT, K2, G);
    return hipGetLastError();
}

}  // namespace ssa
