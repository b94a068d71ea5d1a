// ssa_batch.h -- the persistent many-series kernel (batch.hip): LDS layout,
// limits and launch arguments.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace ssa {

struct BatchArgs {
    int nseries;
    const double* series;      // all series, concatenated (FP64)
    const long long* offs;     // [nseries + 1] start of each series in `series`
    const int* Ls;             // [nseries] window lengths
    const int* ks;             // [nseries] triples per series
    const long long* soff;     // [nseries] start of each series' sigma block
    int d_max, check_every;
    double tol;
    unsigned long long seed;
    double* sigma;             // series s: k_s values at soff[s]
    float* U;                  // series s: L_s x k column-major at uoff[s]
    const long long* uoff;
    float* V;                  // series s: K_s x k column-major at voff[s]
    const long long* voff;
    float* recon;              // series s: k elementary series of N_s at roff[s] (may be null)
    const long long* roff;
    int* info;                 // [nseries * 4]: steps, converged, restarts, DGKS passes
    char* slots;               // one slot of slot_bytes per workgroup
    size_t slot_bytes, o_ab, o_u, o_v, o_scratch, o_p, o_q;
    long long ld;              // leading dimension of the slot's bases
    unsigned* queue;           // work counter, 0 at launch
};

namespace batch {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kEpt = 32;
constexpr int kMaxMp = 10240;  // largest half-length FFT held in LDS (N <= 20480)
constexpr int kTwTab = 128;    // two-level twiddle tables, each <= sqrt(kMaxMp) rounded up
constexpr int kDmax = 320;     // Krylov dimension cap of the batched path
constexpr int kMaxK = 32;      // triples per series
constexpr int kEdge = 512;     // Hankelization entries with <= kEdge terms summed directly
constexpr double kBreakdownTol = 1e-6;
constexpr double kResidFloor = 1e-5;

struct Shared {
    float2 buf[kMaxMp];
    float2 tw_hi[kTwTab];
    float2 tw_lo[kTwTab];
    double red[kWaves][kDmax + 2];
    double h[kDmax + 2];
    double alpha[kDmax + 3];
    double beta[kDmax + 3];
    double tri[2 * (kDmax + 2)];
    double lo[kMaxK], hi[kMaxK], lam[kMaxK], qlast[kMaxK], wprev[kMaxK], resid[kMaxK];
    double xs[kThreads];
    int cnt[kThreads];
    double misc[kWaves];
    int imisc[8];
    FftStages st;
};

}  // namespace batch

hipError_t launch_batch(const BatchArgs& a, int nslots, hipStream_t s);
size_t batch_lds_bytes();

}  // namespace ssa
