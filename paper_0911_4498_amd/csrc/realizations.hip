// realizations.hip -- statistics over repeated realizations of a series
// (Sec. "Bootstrap Confidence Intervals Construction"): the rank-d
// reconstruction G_r of each realization is the sum of its first d elementary
// series; per point n, the mean over realizations, the (R-1)-normalized
// variance and, against a known series, the mean square error.  FP64 sums in a
// fixed order (realizations, then triples).
#include <hip/hip_runtime.h>

#include "ssa_hmatrix.h"

namespace ssa {
namespace rs {

// recon: realization r's elementary series i at recon + (r*d + i)*N
__global__ __launch_bounds__(256) void k_stats(const float* __restrict__ recon, long long R, int d, long long N,
                                               const double* __restrict__ truth, double* __restrict__ mean,
                                               double* __restrict__ var, double* __restrict__ mse) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    double m = 0.0;
    for (long long r = 0; r < R; ++r) {
        double g = 0.0;
        for (int i = 0; i < d; ++i) g += (double)recon[(r * d + i) * N + n];
        m += g;
    }
    m /= (double)R;
    double v = 0.0, e = 0.0;
    const double tn = truth ? truth[n] : 0.0;
    for (long long r = 0; r < R; ++r) {
        double g = 0.0;
        for (int i = 0; i < d; ++i) g += (double)recon[(r * d + i) * N + n];
        v += (g - m) * (g - m);
        e += (g - tn) * (g - tn);
    }
    mean[n] = m;
    var[n] = R > 1 ? v / (double)(R - 1) : 0.0;
    if (truth && mse) mse[n] = e / (double)R;
}

}  // namespace rs

hipError_t launch_realization_stats(const float* recon, long long R, int d, long long N, const double* truth,
                                    double* mean, double* var, double* mse, hipStream_t s) {
    hipLaunchKernelGGL(rs::k_stats, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, recon, R, d, N, truth, mean,
                       var, mse);
    return hipGetLastError();
}

}  // namespace ssa
