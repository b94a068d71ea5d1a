// ssa_internal.h -- shared declarations of the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft_lds.h"
#include "ssa.h"
#include <hip/hip_ext.h>

namespace ssa {

// Timing of one launch by the kernel's own start and end timestamps, the ones a kernel
// profiler reads (events recorded around a launch would also count its dispatch): the
// library's profiler sets these for the next launch of a timed class, and SSA_LAUNCH hands
// them to hipExtLaunchKernelGGL.  Host-thread local; a launch consumes them.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchTiming g_launch_timing;

#define SSA_LAUNCH(kern, grid, block, shmem, stream, ...)                                              \
    do {                                                                                               \
        if (::ssa::g_launch_timing.start) {                                                            \
            const ::ssa::LaunchTiming t_ = ::ssa::g_launch_timing;                                     \
            ::ssa::g_launch_timing = {};                                                               \
            hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, t_.start, t_.stop, 0, __VA_ARGS__); \
        } else {                                                                                       \
            hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                         \
        }                                                                                              \
    } while (0)

// Geometry of the half-length complex FFT used for every real convolution of
// length M: M' = M/2 = M1 * M2 points, "four-step" order.  Pass 1 transforms
// the M2 strided columns (length M1), applies the W_{M'}^{n2 k1} twiddles and
// stores T[k1][n2]; pass 2 transforms rows (length M2), so the spectrum sits
// at T[k1][k2] = Z[k1 + M1 k2] (transposed, never reordered); pass 3 is the
// inverse column pass.  Pointwise products do not care about the order, so
// the spectral operator of the series is stored in the same layout.
struct ConvGeom {
    int M1, M2;
    long long Mp;  // M1 * M2
    long long M;   // 2 * Mp
    int CB;        // columns per workgroup in passes 1 and 3
    int tw_shift;  // W_{M'}^t = tw_hi[t >> tw_shift] * tw_lo[t & mask]
    FftStages st1, st2;
    const float2* tw1;  // W_{M1}^t, t < M1
    const float2* tw2;  // W_{M2}^t, t < M2
    const float2* tw_lo;
    const float2* tw_hi;
    const double* stop = nullptr;  // non-null: the product kernels return at once while *stop != 0
};

// The radix sequences with kernels of their own (FftFixed, fft_lds.h): 200 = 8·5·5 and
// 256 = 8·8·4, the two factors of the tuned split M' = 51200 of N = 1e5 series (the
// schedule tuner's winner and runner-up).  Every other length runs the generic kernels.
using FftPlanA = FftFixed<8, 5, 5>;
using FftPlanB = FftFixed<8, 8, 4>;
// the long-row passes of N = 2^22 .. 2^24 (M1 or M2 = 2048 and 4096)
using FftPlanC = FftFixed<8, 8, 8, 4>;
using FftPlanD = FftFixed<8, 8, 8, 8>;

// pass-1 input modes
enum { IN_REV = 0, IN_SERIES = 1, IN_VECS = 2 };
// pass-3 output modes
enum { OUT_SLICE = 0, OUT_HANKEL = 1 };

// Two-dimensional arrays (2D-SSA) are flattened row by row with row pitch
// `pitch` (= Ny).  A compressed vector of shape rows x width (an Lx x Ly or
// Kx x Ky sub-array, row by row) sits in the padded coordinates at
// r * pitch + c (c < width), zeros elsewhere; pitch = 0 means a plain series.
struct P1In {
    const float* x;      // IN_REV: input vector (w[m] = x[n_in-1-m]), padded length n_in
    long long n_in;
    const double* f;     // IN_SERIES
    long long N;
    const float* U;      // IN_VECS: vector y < nu is U + y*ldu (padded length lenu), else V
    long long ldu, lenu;
    const float* V;
    long long ldv, lenv;
    int nu;
    long long pitch;     // 0: 1D
    int win, wu, wv;     // widths of x, U and V arrays (pitch > 0)
};

struct P3Out {
    float* out;          // OUT_SLICE: out[t] = y[n_in-1+t] - coef*prev[t], t < n_out
    long long n_in, n_out;
    const float* prev;   // may be null
    const double* coef;  // device scalar, may be null
    long long N, L, K;   // OUT_HANKEL: out[y*ldo + m] = y[m] / cnt(m), m < N
    long long ldo;
    long long pitch;     // 0: 1D; else OUT_SLICE keeps t with t % pitch < wout (compressed),
    int wout;            //   OUT_HANKEL divides by cnt_x(m / pitch) cnt_y(m % pitch) with
    long long Nx, Lx, Kx;  // the y-dimension in (pitch, L, K) and the x-dimension here
};

// Segment layout of a Lanczos vector on the fused single-series path.  A vector
// whose natural element i (i < n) is output y[o + i] of a product's inverse FFT
// is stored in the order pass 3 produces it: segment s = 2*n2 + e (n2 < M2,
// e < 2) holds the y indices m = 2*(M2*n1 + n2) + e with n1 = seg_lo + t at slot
// t < S, so the pass-3 workgroup of columns [c0, c0 + CB) owns the contiguous
// slots [2*c0*S, 2*(c0 + CB)*S).  Slots past a segment's count hold zero, so
// inner products over whole segments equal those over the natural vector.  The
// reversed input of the next product maps every pass-1 column onto whole
// segments too (y index m' = N - 1 - m), which lets pass 1 finish the vector.
struct SegLay {
    long long o, n;  // y index of natural element 0; natural length
    int M1, M2;      // the FFT split
    int S;           // slots per segment, a multiple of 4
    long long len;   // stored length 2 * M2 * S
};

__host__ __device__ inline long long seg_lo(const SegLay& l, int n2, int e) {
    const long long a = l.o - 2LL * n2 - e, step = 2LL * l.M2;
    return a <= 0 ? 0 : (a + step - 1) / step;
}

__host__ __device__ inline int seg_count(const SegLay& l, int n2, int e) {
    const long long b = l.o + l.n - 1 - 2LL * n2 - e;
    if (b < 0) return 0;
    long long hi = b / (2LL * l.M2);
    if (hi > l.M1 - 1) hi = l.M1 - 1;
    const long long lo = seg_lo(l, n2, e);
    return hi >= lo ? (int)(hi - lo + 1) : 0;
}

// natural index held by slot t of segment s, or -1 for a padding slot
__host__ __device__ inline long long seg_natural(const SegLay& l, long long s, long long t) {
    const int n2 = (int)(s >> 1), e = (int)(s & 1);
    if (t >= seg_count(l, n2, e)) return -1;
    return 2 * ((long long)l.M2 * (seg_lo(l, n2, e) + t) + n2) + e - l.o;
}

// stored position of natural element i < n
__host__ __device__ inline long long seg_position(const SegLay& l, long long i) {
    const long long m = l.o + i, c = m >> 1;
    const int e = (int)(m & 1), n2 = (int)(c % l.M2);
    return (2LL * n2 + e) * l.S + (c / l.M2 - seg_lo(l, n2, e));
}

struct ReduceArgs {
    double* part;
    int nchunks, pstride, ncols;
    int ncols_bd;       // a fresh direction after a breakdown is made orthogonal to this many
                        // columns (>= ncols; one-sided projects the V side against none)
    float* r;
    long long n;
    const float* basis;
    long long ld;
    double* h;          // out: projection coefficients (ncols)
    double* coef_out;   // out: alpha_j or beta_{j+1} (the B entry)
    double* scale_out;  // out: normalization factor for the new vector
    double* state;      // [0] running max of |B| entries, [1] restarts, [2] DGKS passes
    unsigned long long seed, stream_ctr;
    int track;          // 1: the coefficient is an entry of B (count it in state[0])
    int full;           // 1: the basis already spans the whole space -> zero vector
    int presummed;      // 1: h[0..ncols] already holds the column sums (k_cgs_colsum)
    int* dgks_flag;     // non-null: a second pass is left to the gated launches (flag set to 1)
    const int* gate;    // non-null: the launch does nothing unless *gate != 0
    double tol_bd;      // breakdown threshold relative to state[0]
    int segmented;      // 1: r and the basis are in layout `seg` (a fresh direction fills
    SegLay seg;         //    the natural slots only; padding slots stay zero)
    long long chunk_rows;  // rows per projection workgroup (a multiple of kProjRows); nchunks of them
    double* snap;       // non-null: gets state[1], state[2] once this launch has updated them
    const double* stop; // non-null: the launch does nothing while *stop != 0
};

// Pass 3 of a product fused with the three-term term and the projection partials
// (k_p3_project): r = y - coef * prev in layout lay, part[c * pstride + b] =
// <basis_c, r> over workgroup b's slots for c < ncols and |r|^2 for c = ncols.
struct P3Seg {
    SegLay lay;
    float* r;
    const float* prev;   // same layout as r; may be null (no three-term term)
    const double* coef;  // device scalar (used with prev)
    const float* basis;  // ncols columns, leading dimension ld, layout lay
    long long ld;
    int ncols;
    double* part;
    int pstride;
};

// The update of the previous vector fused with pass 1 of the next product
// (k_p1_update): x = (r - basis h) * scale in layout lay (natural length n = the
// product's input length) is written to out and transformed as the reversed,
// zero-padded input w[m] = x[n - 1 - m].
// The reduction step of the previous half-step folded into the pass-1 update (three
// launches per half-step): every workgroup sums the same partials in the same fixed order
// as the reduction kernel, so all of them reach that kernel's h, B entry and scale bit for
// bit; workgroup 0 publishes the B entry.  A vector that needs a DGKS pass or a fresh
// direction cannot be finished this way: the launch then marks the solve for a restart
// with the reduction as its own launch and writes nothing else.
// Most pass-3 workgroups (partial sums per column) with which each reduction is folded
// into the next pass-1 update, where every workgroup adds all of them.
constexpr int kFoldMaxChunks = 256;
struct FoldRed {
    const double* part;  // part[c * pstride + chunk]: <basis_c, r> for c < ncols, |r|^2 for c = ncols
    int pstride, nchunks;
    double* coef_out;    // the new B entry (alpha_j or beta_{j+1})
    double* bn;          // running max of the B entries in two slots: read bn[par], write bn[par ^ 1]
    int par;
    int track;           // 1: the entry counts in the running max
    int full;            // 1: the basis already spans the whole space (zero vector)
    double tol_bd;       // breakdown threshold relative to the running max
    double* snap;        // non-null: restarts and DGKS passes after this reduction (none on this path)
    double* fail;        // gets kDoneFallback when the restart is needed
    int presummed;       // 1: k_fold_sums has written the column sums to hsum (ncols + 1 doubles)
    double* hsum;
};

struct P1Seg {
    SegLay lay;
    long long N;         // series length: slot of y index m' holds w[N - 1 - m']
    const float* r;
    const float* basis;
    long long ld;
    int ncols;
    const double* h;     // ncols coefficients (device; not read when the reduction is folded in)
    const double* scale; // device scalar (idem)
    float* out;          // stored length lay.len; must not alias r or the ncols columns
    FoldRed fold;        // the folded reduction (fold.part non-null)
};

// Record of the single-series stopping test (doubles, device; the host reads only
// this): header fields, then the k eigenvalues of B_d^T B_d, the Ritz values of the
// previous test and the residual bounds, each kstride long.
enum {
    kChkHavePrev = 0,  // a previous test exists (stability of the Ritz values)
    kChkDone = 1,      // 1 once a test ended the solve; kDoneFallback once a folded
                       // reduction asked for a restart with the reduction as its own launch
    kChkD = 2,         // Lanczos steps d of the deciding test
    kChkConv = 3,      // 1 if the stopping rule held (or the Krylov space was exhausted)
    kChkNonfinite = 4, // 1 if the series holds NaN or Inf
    kChkRestarts = 5,  // breakdown restarts so far
    kChkDgks = 6,      // DGKS second passes so far
    kChkJJ = 7,        // steps of the latest test
    kChkHdr = 8
};
constexpr double kDoneFallback = 2.0;
constexpr double kResidFloorDev = 1e-5;  // residuals of omega_i < 1e-5 omega_1 judged against 1e-5 omega_1

struct LzCheck {
    const double* alpha;  // Algorithm 1 scalars, 1-based: alpha[1..jj+1], beta[2..jj+1]
    const double* beta;
    int jj, k, dcap;      // test on B_jj; k triples; step cap
    long long rmin;       // min(L, K): B is exact once jj reaches it
    double tol;
    double* rec;          // the record (kChkHdr + 3 kstride doubles)
    const double* snap;   // restarts and DGKS passes after the last reduction before the test
    const double* nonfinite;  // nonzero: the series holds NaN/Inf (may be null)
    double* scr;          // 2 kstride + 2 k dstride doubles
    int kstride;
    long long dstride;    // >= jj + 2
};

struct LzRitz {
    const double* alpha;
    const double* beta;
    const double* rec;    // d and the eigenvalues of the deciding test
    int k, kstride;       // P ((d+1) x k) and Q (d x k), row-major, row stride kstride
    long long dstride;
    double* P;
    double* Q;
    double* sigma;        // k values (device)
    double* scr;          // 8 k dstride doubles
};

constexpr int kEdgeCnt = 2048;   // Hankelization entries with <= this many terms are summed directly
constexpr int kProjRows = 1024;  // rows per workgroup in the projection kernel (256 x float4)
constexpr int kProjCols = 8;     // basis columns per workgroup in the projection kernel
constexpr int kProjColsNarrow = 4;    // ... for vectors of at most kProjNarrowChunks row chunks
constexpr int kProjNarrowChunks = 64;
constexpr long long kRitzWideRows = 1LL << 20;  // Ritz rotations of longer vectors use the scalar-load kernel
constexpr int kBisectMinSteps = 48;  // stopping tests on B_d with d >= this use bisection, not QL
constexpr int kProjLongChunks = 8;  // row chunks per projection workgroup for vectors longer than ...
constexpr long long kProjLongRows = 1LL << 20;  // ... this many rows (fewer reductions and partial sums)

// Rows that one projection workgroup sums before its reduction.
inline long long proj_chunk_rows(long long n) {
    return n > kProjLongRows ? (long long)kProjRows * kProjLongChunks : (long long)kProjRows;
}
constexpr int kMaxCols = 2048;   // most basis columns one projection handles
constexpr int kColsumChunks = 256;  // above this many row chunks the column sums get their own launch

// launchers (kernels.hip); each returns hipSuccess or the launch error
hipError_t launch_tables(const ConvGeom& g, float2* tw1, float2* tw2, float2* tw_lo, float2* tw_hi,
                         hipStream_t s);
hipError_t launch_pass1(const ConvGeom& g, int mode, const P1In& in, int nvec, float2* T1,
                        hipStream_t s);
hipError_t launch_pass2_matvec(const ConvGeom& g, const float4* AB, const float2* T1, float2* T2,
                               hipStream_t s);
hipError_t launch_pass2_embed(const ConvGeom& g, const float2* T1, float4* AB, hipStream_t s);
hipError_t launch_pass2_recon(const ConvGeom& g, const float2* T1all, int k, const double* sigma,
                              const int* offs, const int* members, int g0, int ng, float2* T2all,
                              hipStream_t s);
hipError_t launch_pass3(const ConvGeom& g, int mode, const float2* T2, const P3Out& o, int nvec,
                        hipStream_t s);
hipError_t launch_recon_edges(const double* sigma, const float* U, long long ldu, const float* V, long long ldv,
                              const int* offs, const int* members, int ng, long long N, long long L, long long K,
                              float* out, long long ldo, hipStream_t s);
hipError_t launch_recon_edges_2d(const double* sigma, const float* U, long long ldu, const float* V,
                                 long long ldv, const int* offs, const int* members, int ng, long long Nx,
                                 long long Ny, long long Lx, long long Ly, float* out, long long ldo,
                                 hipStream_t s);
hipError_t launch_check_finite(const double* f, long long N, double* flag, hipStream_t s);
hipError_t launch_fill_zero(double* p, long long n, hipStream_t s);
hipError_t launch_start_vector(float* r, long long n, unsigned long long seed, hipStream_t s);
hipError_t launch_cgs_project(const ReduceArgs& a, hipStream_t s);
hipError_t launch_cgs_colsum(const ReduceArgs& a, hipStream_t s);
hipError_t launch_cgs_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_cgs_update(const float* r, const float* basis, long long ld, int ncols,
                             const double* h, const double* scale, float* out, long long n,
                             const int* gate, hipStream_t s);
hipError_t launch_ritz(const float* basis, long long ld, int ncols, const double* P, int k,
                       float* out, long long ldo, long long n, hipStream_t s);
hipError_t launch_p3_project(const ConvGeom& g, const float2* T2, const P3Seg& a, hipStream_t s);
hipError_t launch_p1_update(const ConvGeom& g, const P1Seg& a, float2* T1, hipStream_t s);
hipError_t launch_fold_sums(const FoldRed& f, int ncols, hipStream_t s);
hipError_t launch_start_seg(float* r, const SegLay& lay, unsigned long long seed, hipStream_t s);
hipError_t launch_ritz_seg(const float* basis, long long ld, int ncols, const double* P, int k, float* out,
                           long long ldo, const SegLay& lay, hipStream_t s);
hipError_t set_fused_attributes();
hipError_t launch_lz_check(const LzCheck& a, hipStream_t s);
hipError_t launch_lz_ritz(const LzRitz& a, int d, hipStream_t s);
hipError_t set_lz_attributes();

// Resumable single-series solve on a bound plan without thick restart (api.cpp): begin
// (embed, start vector), advance (up to max_steps Lanczos steps; the stopping test at its
// check points), stopped (a test ended the solve), idle (every step and test enqueued so far
// has run; no waiting), finish (Ritz triples; ends the run).  ssa_truncated_svd runs them
// in a row; the served form advances each long request one check interval per tick.
int run_begin(ssa_plan p, const double* series_dev, int k);

// Host-side resources of a bound plan (pinned staging, events, the check stream).  A plan
// allocates its own at its first bind; a caller that admits and retires many plans lends
// one set instead (plan_lend_host before the bind), so that nothing is allocated or freed
// per plan -- freeing pinned memory can wait for the whole device.
struct PlanHost {
    double* h_scal = nullptr;
    size_t n_scal = 0;
    double* h_flag = nullptr;
    double* h_rec = nullptr;
    size_t n_rec = 0;
    int* h_grp = nullptr;
    size_t n_grp = 0;
    hipEvent_t grp_done = nullptr;
    hipEvent_t chk_ev[2] = {nullptr, nullptr};
    hipEvent_t ab_ev = nullptr, run_ev = nullptr;
    hipStream_t chk_stream = nullptr;
};
int host_alloc(PlanHost& h, size_t n_scal, size_t n_rec, size_t n_grp);
int host_alloc_for(PlanHost& h, int k_max, const ssa_opts* opts);  // enough for any plan with this k_max
void host_free(PlanHost& h);
int plan_lend_host(ssa_plan p, const PlanHost& h);
int run_advance(ssa_plan p, int max_steps);
int run_stopped(ssa_plan p);
int run_idle(ssa_plan p);
int run_finish(ssa_plan p, double* sigma_dev, float* U_dev, float* V_dev, ssa_info* info);
hipError_t set_kernel_attributes();
// set_kernel_attributes() once per process; its result afterwards (api.cpp)
hipError_t kernel_attributes_once();
// The automatic FFT geometry of a 1D plan for a series of length N: the schedule that
// ssa_embed_plan picks without schedule options (twiddle pointers left unset); false when no
// admissible transform length exists (api.cpp).
bool auto_geometry(long long N, ConvGeom* g);

// host small eigen/singular solver (small_svd.cpp)
// Ritz values of the (d+1) x d lower bidiagonal B_d (alpha[1..d] on the
// diagonal, beta[2..d+1] below it; arrays indexed as in Algorithm 1).
// Writes the k largest omega (descending) and their residual bounds
// alpha[d+1] * |P[d, i]| (the last component of the left singular vector).
void bidiag_ritz_values(const double* alpha, const double* beta, int d, int k, double* omega,
                        double* resid, double* work);
// Top-k singular triples of B_d: omega[k], P ((d+1) x k row-major), Q (d x k row-major).
void bidiag_ritz_vectors(const double* alpha, const double* beta, int d, int k, double* omega,
                         double* P, double* Q, double* work);
size_t bidiag_work_doubles(int d);
// Top-k singular triples of a dense nr x nc matrix A (row-major, nr >= nc):
// omega[k] descending, P (nr x k row-major, left vectors), Q (nc x k, right).
// Used for the projected matrix of a restarted bidiagonalization, which is
// no longer bidiagonal.
void dense_ritz(const double* A, int nr, int nc, int k, double* omega, double* P, double* Q);

}  // namespace ssa
