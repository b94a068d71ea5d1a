// ssa_hmatrix.h -- launchers of the structural-change (H-matrix) and
// repeated-realization statistics kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace ssa {

hipError_t launch_hm_windows(const double* f, long long B, long long MB, double* out, hipStream_t s);
hipError_t launch_hm_corr(const double* f, long long N, long long L, const float* U, int k, const int* I, int nI,
                          long long MB, double* c2, hipStream_t s);
hipError_t launch_hm_energy(const double* f, long long N, long long L, double* sq, hipStream_t s);
// prefix-sums c2 (MB rows) and sq in place, then the indices
hipError_t launch_hm_rows(double* c2, double* sq, long long P, long long MB, long long MT, long long K2, double* G,
                          hipStream_t s);

hipError_t launch_realization_stats(const float* recon, long long R, int d, long long N, const double* truth,
                                    double* mean, double* var, double* mse, hipStream_t s);

}  // namespace ssa
