// ssa_batch.h -- the many-series engine (batch.hip): per-series table, LDS
// layout, limits and launch arguments.
//
// A batch advances all of its series in lockstep; every launch has one
// workgroup per series.  A Lanczos half-step is two launches: the FFT product
// of each series in its workgroup's LDS, then its Gram-Schmidt step.  The
// state of a series between launches (spectral operator, Lanczos bases,
// alpha/beta, stopping-test history) lives in its own region of the
// caller's workspace.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace ssa {
namespace batch {

constexpr int kFftThreads = 1024;  // set-up, FFT-product and Hankelization kernels (FFT in LDS)
constexpr int kFftWaves = kFftThreads / 64;
constexpr int kThreads = 512;     // stopping-test and Ritz kernels
constexpr int kWaves = kThreads / 64;
constexpr int kCgsThreads = 512;  // Gram-Schmidt kernel (small LDS)
constexpr int kCgsWaves = kCgsThreads / 64;
constexpr int kCgsCols = 16;      // basis columns per projection pass
constexpr int kEpt = 16;          // points per thread of one LDS FFT stage
constexpr int kMaxMp = 10240;  // largest half-length FFT held in LDS (N <= 20480)
constexpr int kTwTab = 128;    // two-level twiddle tables, each <= sqrt(kMaxMp) rounded up
constexpr int kDmax = 320;     // Krylov dimension cap of the batched path
constexpr int kMaxK = 32;      // triples per series
constexpr int kEdge = 512;     // Hankelization entries with <= kEdge terms summed directly
constexpr double kBreakdownTol = 1e-6;
constexpr double kResidFloor = 1e-5;

// per-series state (doubles at BSeries::o_state)
enum {
    kStBnorm = 0,     // largest alpha/beta so far (breakdown threshold)
    kStRestarts = 1,  // random restarts after a vanishing alpha/beta
    kStDgks = 2,      // second Gram-Schmidt passes
    kStDone = 3,      // 1 once the stopping rule (or the step cap) ended the series
    kStD = 4,         // Lanczos steps d of the final bidiagonal
    kStConv = 5,      // 1 if the stopping rule held
    kStHavePrev = 6,  // a previous check exists (stability test)
    kStJ = 7,         // the series' current Lanczos step j (1 after set-up)
    kStLam = 8,       // k eigenvalues of B_d^T B_d (omega^2), descending
    kStWprev = kStLam + kMaxK,
    kStResid = kStWprev + kMaxK,
    kStDoubles = kStResid + kMaxK
};

}  // namespace batch

// One series of a batch (host-built, uploaded per solve).
struct BSeries {
    const double* f;           // the series (device, N values)
    long long N;
    long long Li, Ki;          // internal window / lag count, Li <= Ki
    long long reg;             // byte offset of the series' region in the workspace
    long long ldu, ldv;        // leading dimensions of the U / V bases (floats)
    double* sigma;             // outputs (device): k values, descending
    float* U;                  // L x k, u_i at + i*L
    float* V;                  // K x k, v_i at + i*K
    float* recon;              // N x k, elementary series i at + i*N (may be null: no Hankelization)
    int* info;                 // 4 ints: steps, converged, restarts, DGKS passes (may be null)
    long long o_ab, o_tw, o_u, o_v, o_r, o_alpha, o_beta, o_state, o_p, o_q, o_scr;  // in the region
    unsigned long long seed;   // start and restart vectors
    int L, k, transposed, dcap;  // user window, triples, L > K, Krylov cap
    int Mp, tw_shift, pad0, pad1;
    FftStages st;              // radix plan of the M'-point complex FFT
};

struct BatchArgs {
    int nseries;               // workgroups of the launch (entries of list, if any)
    const int* list;           // series (table slots) of the launch; null = 0 .. nseries-1
    const BSeries* tab;
    char* ws;                  // workspace base (series regions)
    unsigned* ndone;           // series finished so far (may be null)
    int* done_flags;           // per table slot: 1 once the series is finished (may be null)
    int check_every;
    int onesided;              // 1: the V basis (length Ki) is not reorthogonalized
    double tol;
};

hipError_t launch_batch_init(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_conv(const BatchArgs& a, int side, hipStream_t s);
hipError_t launch_batch_cgs(const BatchArgs& a, int side, hipStream_t s);
hipError_t launch_batch_check(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_ritz(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_hankel(const BatchArgs& a, hipStream_t s);
size_t batch_lds_bytes();

}  // namespace ssa
