// api.cpp -- the C ABI of include/ssa.h: plans, workspace layout, the Lanczos
// driver and the reconstruction.  Every arithmetic step on vectors runs in the
// kernels of kernels.hip; the host only sizes, launches, and solves the small
// (d+1) x d bidiagonal problem that decides when to stop (small_svd.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ssa.h"
#include "ssa_internal.h"

using namespace ssa;

namespace {

constexpr int kMaxFactor = 4096;   // longest single-workgroup FFT (one LDS row)
constexpr int kMaxDmax = 1024;     // Krylov dimension cap supported by the kernels
constexpr double kBreakdownTol = 1e-6;  // relative size of a vanishing alpha/beta (FP32 products)
constexpr double kResidFloor = 1e-5;    // residuals of omega_i < 1e-5 omega_1 are judged against 1e-5 omega_1
constexpr int kMaxGroupBatch = 64;
constexpr int kMaxRestartDmax = 512;  // basis cap of the restarted solver (host dense SVD per cycle)
constexpr int kMaxCycles = 64;        // thick restarts before the solver gives up
constexpr int kGrid2ChunksOneSided = 16;  // one-sided: grid second pass above 16 x 1024 = 16384 rows
// Longest basis vector of the fused path: one workgroup adds the pass-3 partial sums of
// every column, and a DGKS pass in that workgroup must stay short.
constexpr long long kFusedMaxRows = 1LL << 20;
// Columns (with |r|^2) up to which the folded reduction sums the partials inside every
// pass-1 workgroup; beyond, k_fold_sums adds them first.  Measured at N = 1e5: each
// column costs the pass-1 launch about 0.09 us, the extra launch about 8 us with its gap
// (a threshold of 32 or 88 columns made that solve 4% and 2% slower).
constexpr int kFoldInlineCols = 160;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool smooth7(long long n) {
    if (n < 1) return false;
    for (long long p : {2LL, 3LL, 5LL, 7LL})
        while (n % p == 0) n /= p;
    return n == 1;
}

// The most balanced split M' = M1 * M2 (M1 <= M2, both <= kMaxFactor) of a
// 7-smooth M', or 0 if M' has none.
int balanced_m1(long long mp) {
    if (!smooth7(mp)) return 0;
    int best1 = 0;
    for (long long a = 1; a * a <= mp; ++a) {
        if (mp % a) continue;
        const long long b = mp / a;
        if (b > kMaxFactor || a > kMaxFactor) continue;
        best1 = (int)a;  // largest a <= sqrt(mp) that works
    }
    return best1;
}

// Smallest M' >= ceil(N/2) with a split M' = M1 * M2, both 7-smooth and
// <= kMaxFactor; among the splits of that M' the most balanced one (M1 <= M2).
bool choose_fft(long long N, long long& Mp, int& M1, int& M2) {
    for (long long mp = (N + 1) / 2; mp <= (long long)kMaxFactor * kMaxFactor; ++mp) {
        const int best1 = balanced_m1(mp);
        if (best1 > 0) {
            Mp = mp;
            M1 = best1;
            M2 = (int)(mp / best1);
            return true;
        }
    }
    return false;
}

FftStages make_stages(int n) {
    FftStages st{};
    st.n = n;
    int m = n;
    while (m % 8 == 0 && st.nstages < kMaxStages) { st.radix[st.nstages++] = 8; m /= 8; }
    while (m % 4 == 0 && st.nstages < kMaxStages) { st.radix[st.nstages++] = 4; m /= 4; }
    while (m % 2 == 0 && st.nstages < kMaxStages) { st.radix[st.nstages++] = 2; m /= 2; }
    for (int p : {3, 5, 7})
        while (m % p == 0 && st.nstages < kMaxStages) { st.radix[st.nstages++] = p; m /= p; }
    return st;
}

// Columns per workgroup of passes 1 and 3: enough workgroups (~M2/CB >= 256) comes first;
// at N = 1e5 (M1 x M2 = 200 x 250) CB = 1 beats CB = 4 by 10% per product although the
// wider blocks fetch fewer partial lines (measured over every split of M' = 50000).
int default_cb(int M1, int M2) {
    return (int)std::min<long long>({16LL, 8192LL / M1, std::max(1LL, ((long long)M2 + 255) / 256)});
}

// Segment layout of vectors whose natural element i is y index o + i (i < n).
SegLay make_seglay(const ConvGeom& g, long long o, long long n) {
    SegLay l{};
    l.o = o;
    l.n = n;
    l.M1 = g.M1;
    l.M2 = g.M2;
    int smax = 0;
    for (int n2 = 0; n2 < g.M2; ++n2)
        for (int e = 0; e < 2; ++e) smax = std::max(smax, seg_count(l, n2, e));
    l.S = std::max(4, (smax + 3) / 4 * 4);
    l.len = 2LL * g.M2 * l.S;
    return l;
}

void fill_geom(long long Mp, int M1, int M2, int cb, ConvGeom& g) {
    g.M1 = M1;
    g.M2 = M2;
    g.Mp = Mp;
    g.M = 2 * Mp;
    g.CB = std::max(1, cb);
    int shift = 0;
    while ((1LL << (2 * shift)) < Mp) ++shift;
    g.tw_shift = shift;
    g.st1 = make_stages(M1);
    g.st2 = make_stages(M2);
}

}  // namespace

struct ssa_plan_s {
    long long N, L, K;  // as requested (2D: N = Nx Ny, L = Lx Ly, K = Kx Ky)
    int transposed;     // L > K: solved for X^T (window K)
    long long Li, Ki;   // internal window / lag count, Li <= Ki
    int is2d;           // 2D-SSA: an Nx x Ny array with an Lx x Ly window, flattened row by row
    long long Nx, Ny, Lx, Ly, Kx, Ky;
    long long rows[2], width[2];  // shape of the internal U-side (0) and V-side (1) vectors
    int k_max, d_max, check_every;
    int keep;   // thick restart: Ritz pairs kept per cycle (0: no restart)
    int onesided;  // 1: only the length-Li basis (U) is reorthogonalized
    int kcols;  // columns of the P/Q coefficient buffers: max(k_max, keep)
    int fused;  // 1: the fused half-step of fused.hip (three or four launches), bases in the segment layout
    int fold;   // 1: each reduction is folded into the next pass-1 update (three launches)
    int fold_off = 0;  // this solve restarted without the fold (a DGKS pass or a breakdown)
    SegLay layU, layV;  // segment layouts of the U-side (length Li) and V-side (length Ki) vectors
    int nblk;   // pass-3 workgroups of a product (partial sums per column on the fused path)
    double tol;
    unsigned long long seed;
    ConvGeom g;
    long long ldU, ldV;
    int pstride, nchunks_max;
    size_t ws_bytes;
    size_t o_ab, o_tw1, o_tw2, o_twlo, o_twhi, o_t1, o_t2, o_U, o_V, o_r, o_part, o_h, o_sc, o_alpha,
        o_beta, o_state, o_P, o_Q, o_flag, o_grp, o_rt1, o_rt2, o_rot, o_rec, o_lzscr, o_snap;
    int nsnap;         // half-steps with a state snapshot slot (2 doubles each)
    int nrec;          // doubles of the stopping-test record (kChkHdr + 3 kcols)
    long long dstride; // d_max + 2: per-triple length of the device stopping-test scratch
    size_t grp_ints;
    // bound state
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int bound = 0, embedded = 0;
    // pinned host staging
    double* h_scal = nullptr;   // alpha (d_max+3) | beta (d_max+3) | P | Q | sigma
    double* h_flag = nullptr;
    double* h_rec = nullptr;    // two stopping-test records (double-buffered)
    int* h_grp = nullptr;
    hipEvent_t grp_done = nullptr;
    hipEvent_t chk_ev[2] = {nullptr, nullptr};
    // the stopping test runs on its own stream, beside the Lanczos steps
    hipStream_t chk_stream = nullptr;
    hipEvent_t ab_ev = nullptr;  // the scalars of the tested step are written
    const double* stop_dev = nullptr;  // during a fused solve: the test's "done" flag
    // a resumable solve on the device-test path (run_begin .. run_finish)
    struct Run {
        int active = 0, k = 0, j = 1, d_cap = 0;
        int pend_jj = -1, pend_buf = 0, cur_buf = 0, last_chk = -1;
        int steps_run = 0, stopped = 0;
        const double* fin_rec = nullptr;  // pinned copy of the record that ended the solve
    } run;
    hipEvent_t run_ev = nullptr;  // the main stream has run every step enqueued so far
    const ssa::PlanHost* lent = nullptr;  // host resources lent by the caller (not freed here)
    std::vector<double> work;
    // optional per-kernel-class timing (HIP events around the launches of the
    // classes in prof_mask; launch counts and bytes are kept for all classes)
    int prof_on = 0;
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pairs[SSA_PROF_NCLASSES];
    int prof_every = 1;                        // time one launch in prof_every of a timed class
    long long prof_seen[SSA_PROF_NCLASSES] = {};
    double prof_bytes[SSA_PROF_NCLASSES] = {};
    long long prof_count[SSA_PROF_NCLASSES] = {};
};

namespace {

template <typename T>
T* at(ssa_plan p, size_t off) {
    return reinterpret_cast<T*>(p->ws + off);
}

void layout(ssa_plan p) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + bytes, 256);
        return r;
    };
    const ConvGeom& g = p->g;
    const long long S = 1LL << g.tw_shift;
    p->o_ab = take(sizeof(float4) * (size_t)g.Mp);
    p->o_tw1 = take(sizeof(float2) * (size_t)g.M1);
    p->o_tw2 = take(sizeof(float2) * (size_t)g.M2);
    p->o_twlo = take(sizeof(float2) * (size_t)S);
    p->o_twhi = take(sizeof(float2) * (size_t)((g.Mp + S - 1) / S));
    p->o_t1 = take(sizeof(float2) * (size_t)g.Mp);
    p->o_t2 = take(sizeof(float2) * (size_t)g.Mp);
    p->o_U = take(sizeof(float) * (size_t)(p->d_max + 1) * p->ldU);
    p->o_V = take(sizeof(float) * (size_t)(p->d_max + 1) * p->ldV);
    p->o_r = take(sizeof(float) * (size_t)std::max(p->ldU, p->ldV));
    p->o_part = take(sizeof(double) * (size_t)(p->d_max + 2) * p->pstride);
    p->o_h = take(sizeof(double) * (size_t)(p->d_max + 2));
    p->o_sc = take(sizeof(double) * 8);
    p->o_alpha = take(sizeof(double) * (size_t)(p->d_max + 3));
    p->o_beta = take(sizeof(double) * (size_t)(p->d_max + 3));
    p->o_state = take(sizeof(double) * 8);
    p->o_P = take(sizeof(double) * (size_t)(p->d_max + 1) * p->kcols);
    p->o_Q = take(sizeof(double) * (size_t)p->d_max * p->kcols);
    p->o_flag = take(sizeof(int) * 64);
    p->grp_ints = (size_t)(kMaxGroupBatch + 1) + (size_t)kMaxGroupBatch * p->k_max;
    p->o_grp = take(sizeof(int) * p->grp_ints);
    p->o_rt1 = take(sizeof(float2) * (size_t)g.Mp * 2 * p->k_max);
    p->o_rt2 = take(sizeof(float2) * (size_t)g.Mp * kMaxGroupBatch);
    p->o_rot = take(sizeof(float) * (size_t)p->keep * std::max(p->ldU, p->ldV));
    p->nrec = kChkHdr + 3 * p->kcols;
    p->dstride = p->d_max + 2;
    p->o_rec = take(sizeof(double) * (size_t)p->nrec);
    p->o_lzscr = take(sizeof(double) * (8 * (size_t)p->kcols * p->dstride + 2 * (size_t)p->kcols));
    p->nsnap = 2 * p->d_max + 4;
    p->o_snap = take(sizeof(double) * 2 * (size_t)p->nsnap);
    p->ws_bytes = o;
}

ConvGeom bound_geom(ssa_plan p) {
    ConvGeom g = p->g;
    g.tw1 = at<float2>(p, p->o_tw1);
    g.tw2 = at<float2>(p, p->o_tw2);
    g.tw_lo = at<float2>(p, p->o_twlo);
    g.tw_hi = at<float2>(p, p->o_twhi);
    return g;
}

hipEvent_t next_event(ssa_plan p) {
    if (p->ev_next == p->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_next++];
}

// Brackets one launch of kernel class `cls`; `bytes` is the launch's
// algorithmic HBM traffic (what the method must read and write).
struct ProfScope {
    ssa_plan p;
    int cls;
    double bytes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t st;
    // A timed launch gets the kernel's own start and end timestamps when its launcher
    // goes through SSA_LAUNCH (it consumes ssa::g_launch_timing); otherwise the two
    // events bracket the scope on the stream.
    ProfScope(ssa_plan p_, int cls_, double bytes_, hipStream_t st_ = nullptr)
        : p(p_), cls(cls_), bytes(bytes_), st(st_ ? st_ : p_->stream) {
        if (p->prof_on && (p->prof_mask >> cls & 1u) && p->prof_seen[cls]++ % p->prof_every == 0) {
            e0 = next_event(p);
            e1 = e0 ? next_event(p) : nullptr;
            if (e0 && e1) {
                (void)hipEventRecord(e0, st);
                ssa::g_launch_timing = {e0, e1};
            } else {
                e0 = e1 = nullptr;
            }
        }
    }
    ~ProfScope() {
        p->prof_bytes[cls] += bytes;
        p->prof_count[cls] += 1;
        if (p->prof_on && e0) {
            if (ssa::g_launch_timing.start == e0) {  // no launch consumed them
                ssa::g_launch_timing = {};
                (void)hipEventRecord(e1, st);
            }
            p->prof_pairs[cls].push_back({e0, e1});
        }
    }
};

#define SSA_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return SSA_EDEVICE;      \
    } while (0)

// One convolution with the embedded series: out[t] = y[n_in-1+t] - coef*prev[t],
// for an input vector of side `side` (0: U side, 1: V side).  A 2D plan works
// in the padded row-pitch coordinates (n_in = (rows - 1) Ny + width) and
// scatters the input / gathers the output there, so X of 2D-SSA is the
// row/column selection of the 1D Hankel matrix of the flattened array.
int convolve(ssa_plan p, const ConvGeom& g, const float* x, int side, float* out, const float* prev,
             const double* coef) {
    hipStream_t s = p->stream;
    const long long n_in = p->is2d ? (p->rows[side] - 1) * p->Ny + p->width[side] : p->width[side];
    const double len_in = (double)p->rows[side] * p->width[side];
    const double len_out = (double)p->rows[1 - side] * p->width[1 - side];
    P1In in{};
    in.x = x;
    in.n_in = n_in;
    if (p->is2d) {
        in.pitch = p->Ny;
        in.win = (int)p->width[side];
    }
    const double mp = (double)g.Mp;
    {
        ProfScope ps(p, SSA_PROF_PASS1, 4.0 * len_in + 8.0 * mp);
        SSA_TRY(launch_pass1(g, IN_REV, in, 1, at<float2>(p, p->o_t1), s));
    }
    {
        // T1 in (8 B a point), the spectral operator (A, B: 16 B a point), T2 out (8 B)
        ProfScope ps(p, SSA_PROF_PASS2, 32.0 * mp);
        SSA_TRY(launch_pass2_matvec(g, at<float4>(p, p->o_ab), at<float2>(p, p->o_t1), at<float2>(p, p->o_t2), s));
    }
    P3Out o{};
    o.out = out;
    o.n_in = n_in;
    o.n_out = p->N + 1 - n_in;
    o.prev = prev;
    o.coef = coef;
    if (p->is2d) {
        o.pitch = p->Ny;
        o.wout = (int)p->width[1 - side];
    }
    {
        ProfScope ps(p, SSA_PROF_PASS3, 8.0 * mp + 4.0 * len_out * (prev ? 2.0 : 1.0));
        SSA_TRY(launch_pass3(g, OUT_SLICE, at<float2>(p, p->o_t2), o, 1, s));
    }
    return SSA_OK;
}

// Classical Gram-Schmidt of the residual r (length n) against `ncols` basis
// columns, then the normalized vector becomes basis column `out_col` (ncols
// if negative); the B entry goes to *coef_out.
int orthonormalize(ssa_plan p, float* basis, long long ld, int ncols, long long n, double* coef_out, int track,
                   unsigned long long ctr, int out_col = -1, int ncols_bd = -1) {
    hipStream_t s = p->stream;
    float* r = at<float>(p, p->o_r);
    double* h = at<double>(p, p->o_h);
    double* sc = at<double>(p, p->o_sc);
    ReduceArgs a{};
    a.part = at<double>(p, p->o_part);
    a.chunk_rows = proj_chunk_rows(n);
    a.nchunks = (int)((n + a.chunk_rows - 1) / a.chunk_rows);
    a.pstride = p->pstride;
    a.ncols = ncols;
    a.ncols_bd = ncols_bd < ncols ? ncols : ncols_bd;
    a.r = r;
    a.n = n;
    a.basis = basis;
    a.ld = ld;
    a.h = h;
    a.coef_out = coef_out;
    a.scale_out = sc;
    a.state = at<double>(p, p->o_state);
    a.seed = p->seed;
    a.stream_ctr = ctr;
    a.snap = ctr < (unsigned long long)p->nsnap ? at<double>(p, p->o_snap) + 2 * ctr : nullptr;
    a.track = track;
    a.full = ncols >= n ? 1 : 0;
    a.tol_bd = kBreakdownTol;
    {
        ProfScope ps(p, SSA_PROF_DOTS, 4.0 * (double)n * (ncols + 1));
        SSA_TRY(launch_cgs_project(a, s));
    }
    a.presummed = a.nchunks > kColsumChunks ? 1 : 0;
    // A DGKS second pass inside the one-workgroup finish reads the whole basis through one
    // CU: fine while rare and short, ruinous for long vectors (an N = 2^24 pass would take
    // minutes) and for the reorthogonalized side of the one-sided scheme, where it is
    // frequent.  There the finish hands it to four gated launches over the whole grid,
    // which return at once when no second pass was needed.
    const long long grid2_rows = (long long)(p->onesided ? kGrid2ChunksOneSided : kColsumChunks) * kProjRows;
    const bool grid2 = ncols > 0 && n > grid2_rows;
    int* flag2 = at<int>(p, p->o_flag) + 8;
    a.dgks_flag = grid2 ? flag2 : nullptr;
    if (a.presummed) {
        ProfScope ps(p, SSA_PROF_REDUCE, 8.0 * (double)a.nchunks * (ncols + 1));
        SSA_TRY(launch_cgs_colsum(a, s));
    }
    {
        ProfScope ps(p, SSA_PROF_REDUCE, a.presummed ? 8.0 * (ncols + 1) : 8.0 * (double)a.nchunks * (ncols + 1));
        SSA_TRY(launch_cgs_reduce(a, s));
    }
    float* out = basis + (long long)(out_col < 0 ? ncols : out_col) * ld;
    {
        ProfScope ps(p, SSA_PROF_UPDATE, 4.0 * (double)n * (ncols + 2));
        SSA_TRY(launch_cgs_update(r, basis, ld, ncols, h, sc, out, n, nullptr, s));
    }
    if (grid2) {
        // second pass on out = r - basis h (in place), a profiling class of its own: these
        // launches return at once unless the finish asked for the pass, so they would
        // distort the per-launch times of the first-pass classes
        ReduceArgs b = a;
        b.r = out;
        b.dgks_flag = nullptr;
        b.gate = flag2;
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_project(b, s));
        }
        if (b.presummed) {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_colsum(b, s));
        }
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_reduce(b, s));
        }
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_update(out, basis, ld, ncols, h, sc, out, n, flag2, s));
        }
    }
    return SSA_OK;
}

// Reduction step of the fused path: the partial sums in the partials buffer (nchunks
// per column) give h, the new B entry and the normalization (k_cgs_reduce).  Long
// bases hand a DGKS second pass to gated launches over the whole grid, which rewrite
// r in place as r - basis h and redo the projection and the reduction; the next
// pass-1 update then uses whichever h and scale were written last.
int fused_finish(ssa_plan p, const float* basis, long long ld, int ncols, int ncols_bd, const SegLay& lay,
                 int nchunks, double* coef_out, int track, unsigned long long ctr) {
    hipStream_t s = p->stream;
    float* r = at<float>(p, p->o_r);
    double* h = at<double>(p, p->o_h);
    double* sc = at<double>(p, p->o_sc);
    ReduceArgs a{};
    a.part = at<double>(p, p->o_part);
    a.nchunks = nchunks;
    a.pstride = p->pstride;
    a.ncols = ncols;
    a.ncols_bd = std::max(ncols, ncols_bd);
    a.r = r;
    a.n = lay.len;
    a.basis = basis;
    a.ld = ld;
    a.h = h;
    a.coef_out = coef_out;
    a.scale_out = sc;
    a.state = at<double>(p, p->o_state);
    a.seed = p->seed;
    a.stream_ctr = ctr;
    a.snap = ctr < (unsigned long long)p->nsnap ? at<double>(p, p->o_snap) + 2 * ctr : nullptr;
    a.track = track;
    a.full = ncols >= lay.n ? 1 : 0;
    a.tol_bd = kBreakdownTol;
    a.segmented = 1;
    a.seg = lay;
    a.presummed = nchunks > kColsumChunks ? 1 : 0;
    a.stop = p->stop_dev;
    const long long grid2_rows = (long long)(p->onesided ? kGrid2ChunksOneSided : kColsumChunks) * kProjRows;
    const bool grid2 = ncols > 0 && lay.n > grid2_rows;
    int* flag2 = at<int>(p, p->o_flag) + 8;
    a.dgks_flag = grid2 ? flag2 : nullptr;
    if (a.presummed) {
        ProfScope ps(p, SSA_PROF_REDUCE, 8.0 * (double)nchunks * (ncols + 1));
        SSA_TRY(launch_cgs_colsum(a, s));
    }
    {
        ProfScope ps(p, SSA_PROF_REDUCE, a.presummed ? 8.0 * (ncols + 1) : 8.0 * (double)nchunks * (ncols + 1));
        SSA_TRY(launch_cgs_reduce(a, s));
    }
    if (grid2) {
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_update(r, basis, ld, ncols, h, sc, r, lay.len, flag2, s));
        }
        ReduceArgs b = a;
        b.dgks_flag = nullptr;
        b.gate = flag2;
        b.chunk_rows = proj_chunk_rows(lay.len);
        b.nchunks = (int)((lay.len + b.chunk_rows - 1) / b.chunk_rows);
        b.presummed = b.nchunks > kColsumChunks ? 1 : 0;
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_project(b, s));
        }
        if (b.presummed) {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_colsum(b, s));
        }
        {
            ProfScope ps(p, SSA_PROF_DGKS2, 0.0);
            SSA_TRY(launch_cgs_reduce(b, s));
        }
    }
    return SSA_OK;
}

// The reduction folded into the next pass-1 update: the partials of the last pass 3
// (against ncols columns) give the B entry coef_out; ctr numbers the reduction as
// fused_finish does.
FoldRed fold_args(ssa_plan p, int ncols, const SegLay& lay, double* coef_out, unsigned long long ctr) {
    FoldRed f{};
    f.part = at<double>(p, p->o_part);
    f.pstride = p->pstride;
    f.nchunks = p->nblk;
    f.coef_out = coef_out;
    f.bn = at<double>(p, p->o_state) + 4;
    f.par = (int)(ctr & 1);
    f.track = 1;
    f.full = ncols >= lay.n ? 1 : 0;
    f.tol_bd = kBreakdownTol;
    f.snap = ctr < (unsigned long long)p->nsnap ? at<double>(p, p->o_snap) + 2 * ctr : nullptr;
    f.fail = at<double>(p, p->o_rec) + kChkDone;
    // many columns: their sums run as a launch of their own (k_fold_sums), which costs less
    // than every pass-1 workgroup fetching all partials
    f.presummed = ncols + 1 > kFoldInlineCols ? 1 : 0;
    f.hsum = at<double>(p, p->o_h);
    return f;
}

// One product of the fused path, first launch: pass 1 finishes x (the previous
// half-step's vector, layout lin, written to out_col; with fold, after the reduction
// that gives its h and scale) and transforms it.
int fused_pass1(ssa_plan p, const ConvGeom& g, const SegLay& lin, const float* basis_in, long long ld_in,
                int ncols_in, float* out_col, const FoldRed* fold) {
    hipStream_t s = p->stream;
    float* r = at<float>(p, p->o_r);
    float2* T1 = at<float2>(p, p->o_t1);
    const double mp = (double)g.Mp;
    P1Seg a{};
    a.lay = lin;
    a.N = p->N;
    a.r = r;
    a.basis = basis_in;
    a.ld = ld_in;
    a.ncols = ncols_in;
    a.h = at<double>(p, p->o_h);
    a.scale = at<double>(p, p->o_sc);
    a.out = out_col;
    if (fold) a.fold = *fold;
    if (fold && fold->presummed) {
        ProfScope ps(p, SSA_PROF_REDUCE, 8.0 * (double)(ncols_in + 1) * fold->nchunks);
        SSA_TRY(launch_fold_sums(*fold, ncols_in, s));
    }
    {
        const double red = fold ? 8.0 * (double)(ncols_in + 1) * (fold->presummed ? 1 : fold->nchunks) : 0.0;
        ProfScope ps(p, SSA_PROF_PASS1, 4.0 * (double)lin.n * (ncols_in + 2) + 8.0 * mp + red);
        SSA_TRY(launch_p1_update(g, a, T1, s));
    }
    return SSA_OK;
}

// The rest of the product: pass 2; pass 3 writes r = y - coef * prev in layout lout and
// the projection partials against ncols_out columns of basis_out.
int fused_pass23(ssa_plan p, const ConvGeom& g, const SegLay& lout, const float* prev, const double* coef,
                 const float* basis_out, long long ld_out, int ncols_out) {
    hipStream_t s = p->stream;
    float* r = at<float>(p, p->o_r);
    float2* T1 = at<float2>(p, p->o_t1);
    float2* T2 = at<float2>(p, p->o_t2);
    const double mp = (double)g.Mp;
    {
        ProfScope ps(p, SSA_PROF_PASS2, 32.0 * mp);  // T1, the operator (16 B a point), T2
        SSA_TRY(launch_pass2_matvec(g, at<float4>(p, p->o_ab), T1, T2, s));
    }
    P3Seg b{};
    b.lay = lout;
    b.r = r;
    b.prev = prev;
    b.coef = coef;
    b.basis = basis_out;
    b.ld = ld_out;
    b.ncols = ncols_out;
    b.part = at<double>(p, p->o_part);
    b.pstride = p->pstride;
    {
        ProfScope ps(p, SSA_PROF_PASS3, 8.0 * mp + 4.0 * (double)lout.n * (ncols_out + (prev ? 2 : 1)));
        SSA_TRY(launch_p3_project(g, T2, b, s));
    }
    return SSA_OK;
}

int check_series(ssa_plan p, const double* series_dev) {
    double* dflag = at<double>(p, p->o_flag);
    SSA_TRY(launch_fill_zero(dflag, 1, p->stream));
    SSA_TRY(launch_check_finite(series_dev, p->N, dflag, p->stream));
    SSA_TRY(hipMemcpyAsync(p->h_flag, dflag, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    SSA_TRY(hipStreamSynchronize(p->stream));
    return *p->h_flag != 0.0 ? SSA_ENONFINITE : SSA_OK;
}

// The spectral operator of the series (Algorithm 2, steps 1-2).  With sync_check the
// series is first checked for NaN/Inf on the device and the host waits for the
// answer; without it the check only leaves its flag in the workspace (the device
// stopping test reports it), so nothing waits.
int do_embed(ssa_plan p, const double* series_dev, bool sync_check = true) {
    if (sync_check) {
        const int rc = check_series(p, series_dev);
        if (rc != SSA_OK) return rc;
    } else {
        double* dflag = at<double>(p, p->o_flag);
        SSA_TRY(launch_fill_zero(dflag, 1, p->stream));
        SSA_TRY(launch_check_finite(series_dev, p->N, dflag, p->stream));
    }
    const ConvGeom g = bound_geom(p);
    P1In in{};
    in.f = series_dev;
    in.N = p->N;
    {
        ProfScope ps(p, SSA_PROF_EMBED, 8.0 * p->N + 8.0 * g.Mp);
        SSA_TRY(launch_pass1(g, IN_SERIES, in, 1, at<float2>(p, p->o_t1), p->stream));
    }
    {
        ProfScope ps(p, SSA_PROF_EMBED, 24.0 * g.Mp);
        SSA_TRY(launch_pass2_embed(g, at<float2>(p, p->o_t1), at<float4>(p, p->o_ab), p->stream));
    }
    p->embedded = 1;
    return SSA_OK;
}

// One half of Lanczos step j (Algorithm 1).  The V half finishes u_j, forms r_j = X^T u_j -
// beta_j v_{j-1}, orthogonalizes it against V (Sec. 3.2.2) and yields alpha_j; the U half
// finishes v_j, forms p_j = X v_j - alpha_j u_j, orthogonalizes it against U and yields
// beta_{j+1}.  gl is the geometry of the fused products (it may carry the early-exit
// flag), g that of the unfused ones.
//
// On the folded path the reduction of each half-step runs inside the next one's pass-1
// launch (not after the V half of step 1, whose pass 1 follows the start vector's own
// reduction).  part 1 enqueues only that launch, part 2 the rest, 0 both: alpha_j comes
// from the U half's first launch, and a stopping test of step j waits for it.
int half_step(ssa_plan p, const ConvGeom& gl, const ConvGeom& g, int j, bool vhalf, int part = 0) {
    float* U = at<float>(p, p->o_U);
    float* V = at<float>(p, p->o_V);
    float* r = at<float>(p, p->o_r);
    double* alpha = at<double>(p, p->o_alpha);
    double* beta = at<double>(p, p->o_beta);
    const long long Li = p->Li, Ki = p->Ki;
    // one-sided: V (length Ki >= Li) keeps only the three-term recurrence of pass 3
    const int ncv = p->onesided ? 0 : j - 1;
    int rc;
    const bool folding = p->fused && p->fold && !p->fold_off;
    if (vhalf) {
        if (p->fused) {
            // finish u_j (folded: after the reduction that yields beta_j); r_j = X^T u_j -
            // beta_j v_{j-1}; its partials against V_{j-1}; alpha_j
            if (part != 2) {
                FoldRed f{};
                if (folding && j >= 2) f = fold_args(p, j - 1, p->layU, beta + j, 2ULL * j - 1);
                rc = fused_pass1(p, gl, p->layU, U, p->ldU, j - 1, U + (long long)(j - 1) * p->ldU,
                                 f.part ? &f : nullptr);
                if (rc != SSA_OK) return rc;
            }
            if (part == 1) return SSA_OK;
            rc = fused_pass23(p, gl, p->layV, j >= 2 ? V + (long long)(j - 2) * p->ldV : nullptr, beta + j, V,
                              p->ldV, ncv);
            if (rc != SSA_OK) return rc;
            if (!folding) rc = fused_finish(p, V, p->ldV, ncv, j - 1, p->layV, p->nblk, alpha + j, 1, 2ULL * j);
        } else {
            // r_j = X^T u_j - beta_j v_{j-1};  alpha_j = |r_j|;  v_j = r_j / alpha_j  (with FRO)
            rc = convolve(p, g, U + (long long)(j - 1) * p->ldU, 0, r,
                          j >= 2 ? V + (long long)(j - 2) * p->ldV : nullptr, beta + j);
            if (rc != SSA_OK) return rc;
            rc = orthonormalize(p, V, p->ldV, ncv, Ki, alpha + j, 1, 2ULL * j, j - 1, j - 1);
        }
        if (rc != SSA_OK) return rc;
    } else {
        if (p->fused) {
            // finish v_j (folded: after the reduction that yields alpha_j); p_j = X v_j -
            // alpha_j u_j; its partials against U_j; beta_{j+1}
            if (part != 2) {
                FoldRed f{};
                if (folding) f = fold_args(p, ncv, p->layV, alpha + j, 2ULL * j);
                rc = fused_pass1(p, gl, p->layV, V, p->ldV, ncv, V + (long long)(j - 1) * p->ldV,
                                 f.part ? &f : nullptr);
                if (rc != SSA_OK) return rc;
            }
            if (part == 1) return SSA_OK;
            rc = fused_pass23(p, gl, p->layU, U + (long long)(j - 1) * p->ldU, alpha + j, U, p->ldU, j);
            if (rc != SSA_OK) return rc;
            if (!folding) rc = fused_finish(p, U, p->ldU, j, j, p->layU, p->nblk, beta + j + 1, 1, 2ULL * j + 1);
        } else {
            // p_j = X v_j - alpha_j u_j;  beta_{j+1} = |p_j|;  u_{j+1} = p_j / beta_{j+1}
            rc = convolve(p, g, V + (long long)(j - 1) * p->ldV, 1, r, U + (long long)(j - 1) * p->ldU, alpha + j);
            if (rc != SSA_OK) return rc;
            rc = orthonormalize(p, U, p->ldU, j, Li, beta + j + 1, 1, 2ULL * j + 1);
        }
        if (rc != SSA_OK) return rc;
    }
    return SSA_OK;
}

// Algorithm 1, first line: u_1 = p_0 / |p_0| with a seeded Gaussian p_0 (the fused
// path leaves u_1 = r * scale to the first pass-1 update); beta_1 = |p_0|.
int start_vector(ssa_plan p) {
    hipStream_t s = p->stream;
    float* U = at<float>(p, p->o_U);
    float* r = at<float>(p, p->o_r);
    double* beta = at<double>(p, p->o_beta);
    const long long Li = p->Li;
    int rc;
    if (p->fused) {
        SSA_TRY(launch_start_seg(r, p->layU, p->seed, s));
        ReduceArgs a0{};
        a0.part = at<double>(p, p->o_part);
        a0.chunk_rows = proj_chunk_rows(p->layU.len);
        a0.nchunks = (int)((p->layU.len + a0.chunk_rows - 1) / a0.chunk_rows);
        a0.pstride = p->pstride;
        a0.r = r;
        a0.n = p->layU.len;
        a0.basis = U;
        a0.ld = p->ldU;
        {
            ProfScope ps(p, SSA_PROF_DOTS, 4.0 * (double)Li);
            SSA_TRY(launch_cgs_project(a0, s));
        }
        rc = fused_finish(p, U, p->ldU, 0, 0, p->layU, a0.nchunks, beta + 1, 0, 1);
    } else {
        SSA_TRY(launch_start_vector(r, Li, p->seed, s));
        rc = orthonormalize(p, U, p->ldU, 0, Li, beta + 1, 0, 1);
    }
    if (rc != SSA_OK) return rc;
    return SSA_OK;
}

// Pinned doubles of a plan's scalar staging (alpha, beta, P, Q, sigma of the host-test path).
size_t host_scal_doubles(int d_max, int kcols, int k_max) {
    return 4 * (size_t)(d_max + 3) + (size_t)(2 * d_max + 1) * kcols + k_max + 8;
}

void use_host(ssa_plan p, const ssa::PlanHost& h) {
    p->h_scal = h.h_scal;
    p->h_flag = h.h_flag;
    p->h_rec = h.h_rec;
    p->h_grp = h.h_grp;
    p->grp_done = h.grp_done;
    p->chk_ev[0] = h.chk_ev[0];
    p->chk_ev[1] = h.chk_ev[1];
    p->ab_ev = h.ab_ev;
    p->run_ev = h.run_ev;
    p->chk_stream = h.chk_stream;
}

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

}  // namespace

namespace ssa {

hipError_t kernel_attributes_once() {
    std::call_once(g_attr_once, [] {
        g_attr_err = set_kernel_attributes();
        const hipError_t e2 = set_fused_attributes();
        if (g_attr_err == hipSuccess) g_attr_err = e2;
        const hipError_t e3 = set_lz_attributes();
        if (g_attr_err == hipSuccess) g_attr_err = e3;
    });
    return g_attr_err;
}

bool auto_geometry(long long N, ConvGeom* g) {
    long long Mp;
    int M1, M2;
    if (!choose_fft(N, Mp, M1, M2)) return false;
    fill_geom(Mp, M1, M2, default_cb(M1, M2), *g);
    return true;
}

}  // namespace ssa

namespace ssa {

// A solve on the device-test path (plans without thick restart), in resumable pieces:
// run_begin embeds the series and enqueues the start vector; run_advance enqueues up to
// max_steps Lanczos steps, launching the stopping test at its check points (on the check
// stream) and waiting for the previous test's record at each; run_finish enqueues the Ritz
// triples once a test has ended the solve.  ssa_truncated_svd runs the three in a row; the
// served form advances many of them a check interval per tick.
int host_alloc(PlanHost& h, size_t n_scal, size_t n_rec, size_t n_grp) {
    h.n_scal = n_scal;
    h.n_rec = n_rec;
    h.n_grp = n_grp;
    if (hipHostMalloc((void**)&h.h_scal, sizeof(double) * n_scal, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.h_flag, sizeof(double) * 16, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.h_rec, sizeof(double) * n_rec, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.h_grp, sizeof(int) * n_grp, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&h.grp_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h.chk_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h.chk_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h.ab_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h.run_ev, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&h.chk_stream, hipStreamNonBlocking) != hipSuccess)
        return SSA_EDEVICE;
    return SSA_OK;
}

void host_free(PlanHost& h) {
    if (h.chk_stream) {
        (void)hipStreamSynchronize(h.chk_stream);
        (void)hipStreamDestroy(h.chk_stream);
    }
    if (h.grp_done) {
        (void)hipEventSynchronize(h.grp_done);
        (void)hipEventDestroy(h.grp_done);
    }
    for (hipEvent_t e : {h.chk_ev[0], h.chk_ev[1], h.ab_ev, h.run_ev})
        if (e) (void)hipEventDestroy(e);
    if (h.h_scal) (void)hipHostFree(h.h_scal);
    if (h.h_flag) (void)hipHostFree(h.h_flag);
    if (h.h_rec) (void)hipHostFree(h.h_rec);
    if (h.h_grp) (void)hipHostFree(h.h_grp);
    h = PlanHost{};
}

int host_alloc_for(PlanHost& h, int k_max, const ssa_opts* opts) {
    const int d_max = std::min(opts && opts->d_max > 0 ? opts->d_max : 8 * k_max + 32, kMaxDmax);
    const int kcols = std::max(k_max, opts ? opts->restart_keep : 0);
    const size_t grp = (size_t)(kMaxGroupBatch + 1) + (size_t)kMaxGroupBatch * k_max;
    return host_alloc(h, host_scal_doubles(d_max, kcols, k_max), 2 * (size_t)(kChkHdr + 3 * kcols), grp);
}

int plan_lend_host(ssa_plan p, const PlanHost& h) {
    if (!p || p->h_scal || !h.h_scal) return SSA_ESTATE;  // before the plan's first bind
    if (host_scal_doubles(p->d_max, p->kcols, p->k_max) > h.n_scal || 2 * (size_t)p->nrec > h.n_rec ||
        p->grp_ints > h.n_grp)
        return SSA_ENOMEM;
    use_host(p, h);
    p->lent = &h;
    return SSA_OK;
}

int run_begin(ssa_plan p, const double* series_dev, int k) {
    int rc = do_embed(p, series_dev, false);
    if (rc != SSA_OK) return rc;
    hipStream_t s = p->stream;
    double* rec = at<double>(p, p->o_rec);
    SSA_TRY(launch_fill_zero(rec, p->nrec, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_alpha), p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_beta), p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_state), 8, s));
    p->fold_off = 0;
    rc = start_vector(p);
    if (rc != SSA_OK) return rc;
    p->run = decltype(p->run){};
    p->run.active = 1;
    p->run.k = k;
    p->run.d_cap = (int)std::min<long long>(p->d_max, std::min(p->Li, p->Ki));
    // Steps enqueued after the deciding test (the host learns of it one test later) do
    // no work on the fused path: its product and reduction kernels return at once once
    // the test's record says done.  Those steps only write columns and scalars past d.
    p->stop_dev = p->fused ? rec + kChkDone : nullptr;
    SSA_TRY(hipEventRecord(p->run_ev, s));
    return SSA_OK;
}

// A folded reduction met a DGKS pass or a breakdown (the record says kDoneFallback; every
// launch after it returned at once): the solve starts over, same start vector, with the
// reduction as its own launch.  Nothing waits on the host.
int run_restart_unfolded(ssa_plan p) {
    auto& R = p->run;
    hipStream_t s = p->stream;
    // the tests enqueued so far read and write the record: the reset comes after them
    if (R.last_chk >= 0) SSA_TRY(hipStreamWaitEvent(s, p->chk_ev[R.last_chk], 0));
    double* rec = at<double>(p, p->o_rec);
    SSA_TRY(launch_fill_zero(rec, p->nrec, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_alpha), p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_beta), p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_state), 8, s));
    p->fold_off = 1;
    const int rc = start_vector(p);
    if (rc != SSA_OK) return rc;
    R.j = 1;
    R.pend_jj = -1;
    R.steps_run = 0;
    R.stopped = 0;
    R.fin_rec = nullptr;
    return SSA_OK;
}

int run_advance(ssa_plan p, int max_steps) {
    auto& R = p->run;
    if (!R.active) return SSA_ESTATE;
    hipStream_t s = p->stream;
    const ConvGeom g = bound_geom(p);
    ConvGeom gl = g;
    gl.stop = p->stop_dev;
    const long long Li = p->Li, Ki = p->Ki;
    double* rec = at<double>(p, p->o_rec);
    double* alpha = at<double>(p, p->o_alpha);
    double* beta = at<double>(p, p->o_beta);
    const int k = R.k;
    for (int n = 0; n < max_steps && !R.stopped; ++n) {
        const int j = R.j;
        const bool folding = p->fused && p->fold && !p->fold_off;
        int rc = half_step(p, gl, g, j, true);
        if (rc != SSA_OK) return rc;
        const int jj = j - 1;
        R.steps_run = jj;
        bool stop = false;
        double done = 0.0;
        const bool test = jj >= k && (jj % p->check_every == 0 || jj >= R.d_cap);
        if (test && folding) {
            // alpha_j and the snapshot of its reduction come from the U half's first launch
            rc = half_step(p, gl, g, j, false, 1);
            if (rc != SSA_OK) return rc;
        }
        if (test) {
            // the test of one check point runs on the check stream, beside the next
            // Lanczos steps (it reads only alpha/beta up to this step and the state
            // snapshot of this step's reduction); the host reads its record one check
            // point later
            SSA_TRY(hipEventRecord(p->ab_ev, s));
            SSA_TRY(hipStreamWaitEvent(p->chk_stream, p->ab_ev, 0));
            LzCheck c{};
            c.alpha = alpha;
            c.beta = beta;
            c.jj = jj;
            c.k = k;
            c.dcap = R.d_cap;
            c.rmin = std::min(Li, Ki);
            c.tol = p->tol;
            c.rec = rec;
            c.snap = at<double>(p, p->o_snap) + 2 * (2 * (long long)j);  // the V half of step j
            c.nonfinite = at<double>(p, p->o_flag);
            c.scr = at<double>(p, p->o_lzscr);
            c.kstride = p->kcols;
            c.dstride = p->dstride;
            {
                ProfScope ps(p, SSA_PROF_CHECK, 16.0 * (jj + 2), p->chk_stream);
                SSA_TRY(launch_lz_check(c, p->chk_stream));
            }
            double* hr = p->h_rec + (size_t)R.cur_buf * p->nrec;
            SSA_TRY(hipMemcpyAsync(hr, rec, sizeof(double) * p->nrec, hipMemcpyDeviceToHost, p->chk_stream));
            SSA_TRY(hipEventRecord(p->chk_ev[R.cur_buf], p->chk_stream));
            R.last_chk = R.cur_buf;
            if (R.pend_jj >= 0) {
                SSA_TRY(hipEventSynchronize(p->chk_ev[R.pend_buf]));
                done = p->h_rec[(size_t)R.pend_buf * p->nrec + kChkDone];
                stop = done != 0.0;
            }
            if (!stop) {
                R.pend_jj = jj;
                R.pend_buf = R.cur_buf;
                R.cur_buf ^= 1;
                if (jj >= R.d_cap) {
                    SSA_TRY(hipEventSynchronize(p->chk_ev[R.pend_buf]));
                    done = p->h_rec[(size_t)R.pend_buf * p->nrec + kChkDone];
                    stop = done != 0.0;
                }
            }
            if (stop) R.fin_rec = p->h_rec + (size_t)R.pend_buf * p->nrec;
        }
        if (stop && done == kDoneFallback) {
            rc = run_restart_unfolded(p);
            if (rc != SSA_OK) return rc;
            continue;
        }
        if (stop) {
            R.stopped = 1;
            break;
        }
        rc = half_step(p, gl, g, j, false, test && folding ? 2 : 0);
        if (rc != SSA_OK) return rc;
        R.j = j + 1;
    }
    SSA_TRY(hipEventRecord(p->run_ev, s));
    return SSA_OK;
}

int run_stopped(ssa_plan p) { return p->run.stopped; }

// Every step and test enqueued so far has finished (no waiting).
int run_idle(ssa_plan p) {
    if (hipEventQuery(p->run_ev) != hipSuccess) return 0;
    if (p->run.last_chk >= 0 && hipEventQuery(p->chk_ev[p->run.last_chk]) != hipSuccess) return 0;
    return 1;
}

// The Ritz triples of a stopped run (stream-ordered: the call returns once they are
// enqueued).  Also ends the run.
int run_finish(ssa_plan p, double* sigma_dev, float* U_dev, float* V_dev, ssa_info* info) {
    auto& R = p->run;
    if (!R.active || !R.stopped) return SSA_ESTATE;
    R.active = 0;
    p->stop_dev = nullptr;
    hipStream_t s = p->stream;
    const int k = R.k;
    const long long Li = p->Li, Ki = p->Ki;
    float* U = at<float>(p, p->o_U);
    float* V = at<float>(p, p->o_V);
    double* rec = at<double>(p, p->o_rec);
    double* alpha = at<double>(p, p->o_alpha);
    double* beta = at<double>(p, p->o_beta);
    double* dP = at<double>(p, p->o_P);
    double* dQ = at<double>(p, p->o_Q);
    float* Uo = p->transposed ? V_dev : U_dev;  // internal U has length Li
    float* Vo = p->transposed ? U_dev : V_dev;
    // Stream-ordered from here: the Ritz coefficients and vectors are enqueued and the
    // call returns; the outputs are complete when the stream has run them.  Everything
    // after this reads the record and the test's scratch, and the next solve rewrites
    // them: order the main stream after every test enqueued.
    SSA_TRY(hipStreamWaitEvent(s, p->chk_ev[R.last_chk], 0));
    if (R.fin_rec[kChkNonfinite] != 0.0) {
        p->embedded = 0;  // the operator holds the non-finite series: unusable
        return SSA_ENONFINITE;
    }
    const int d = (int)R.fin_rec[kChkD];
    const bool conv = R.fin_rec[kChkConv] != 0.0;
    LzRitz rz{};
    rz.alpha = alpha;
    rz.beta = beta;
    rz.rec = rec;
    rz.k = k;
    rz.kstride = k;
    rz.dstride = p->dstride;
    rz.P = dP;
    rz.Q = dQ;
    rz.sigma = sigma_dev;
    rz.scr = at<double>(p, p->o_lzscr);
    {
        ProfScope ps(p, SSA_PROF_CHECK, 16.0 * (d + 2));
        SSA_TRY(launch_lz_ritz(rz, d, s));
    }
    {
        ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Li * (d + 1 + k));
        if (p->fused)
            SSA_TRY(launch_ritz_seg(U, p->ldU, d + 1, dP, k, Uo, Li, p->layU, s));
        else
            SSA_TRY(launch_ritz(U, p->ldU, d + 1, dP, k, Uo, Li, Li, s));
    }
    {
        ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Ki * (d + k));
        if (p->fused)
            SSA_TRY(launch_ritz_seg(V, p->ldV, d, dQ, k, Vo, Ki, p->layV, s));
        else
            SSA_TRY(launch_ritz(V, p->ldV, d, dQ, k, Vo, Ki, Ki, s));
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->steps = d;
        info->converged = conv ? 1 : 0;
        info->restarts = (int)R.fin_rec[kChkRestarts];
        info->dgks_passes = (int)R.fin_rec[kChkDgks];
        info->steps_run = R.steps_run;
        info->half_step_launches = !p->fused ? 6 : (p->fold && !p->fold_off) ? 3 : 4;
        const double* resid = R.fin_rec + kChkHdr + 2 * p->kcols;
        for (int i = 0; i < k && i < 64; ++i) info->resid[i] = resid[i];
    }
    const int status = !conv ? SSA_WARN_NOT_CONVERGED : R.fin_rec[kChkRestarts] > 0.0 ? SSA_WARN_BREAKDOWN : SSA_OK;
    if (info) info->status = status;
    return status;
}

}  // namespace ssa

extern "C" {

// A plan for a series of N values whose trajectory matrix is L x K; for 2D
// plans (is2d) N = Nx Ny, L = Lx Ly, K = Kx Ky.
static int plan_create(long long N, long long L, long long K, int is2d, long long Nx, long long Ny, long long Lx,
                       long long Ly, int k_max, const ssa_opts* opts, size_t* workspace_bytes, ssa_plan* out) {
    const long long r = std::min(L, K);
    if (k_max < 1 || k_max > r || k_max > 256) return SSA_EINVAL;
    ssa_plan p = new (std::nothrow) ssa_plan_s();
    if (!p) return SSA_EINVAL;
    p->N = N;
    p->L = L;
    p->K = K;
    p->transposed = L > K ? 1 : 0;
    p->Li = std::min(L, K);
    p->Ki = std::max(L, K);
    p->is2d = is2d;
    if (is2d) {
        p->Nx = Nx;
        p->Ny = Ny;
        p->Lx = Lx;
        p->Ly = Ly;
        p->Kx = Nx - Lx + 1;
        p->Ky = Ny - Ly + 1;
        // internal window: the smaller of the two shapes (the transpose uses window Kx x Ky)
        const int sL = p->transposed ? 1 : 0;
        p->rows[sL] = Lx;
        p->width[sL] = Ly;
        p->rows[1 - sL] = p->Kx;
        p->width[1 - sL] = p->Ky;
    } else {
        p->rows[0] = p->rows[1] = 1;
        p->width[0] = p->Li;
        p->width[1] = p->Ki;
    }
    p->k_max = k_max;
    int d_max = opts && opts->d_max > 0 ? opts->d_max : 8 * k_max + 32;
    d_max = (int)std::min<long long>({(long long)d_max, r, (long long)kMaxDmax});
    if (d_max < k_max) d_max = k_max;
    p->d_max = d_max;
    p->check_every = opts && opts->check_every > 0 ? opts->check_every : 4;
    p->tol = opts && opts->tol > 0.0 ? opts->tol : 1e-8;
    p->seed = opts && opts->seed ? opts->seed : 1ULL;
    p->keep = 0;
    if (opts && opts->restart_keep > 0) {
        // the whole Krylov space fits under the cap: no restart is ever needed
        if (opts->restart_keep < k_max || (d_max < r && (opts->restart_keep + 2 > d_max || d_max > kMaxRestartDmax))) {
            delete p;
            return SSA_EINVAL;
        }
        if (d_max < r) p->keep = opts->restart_keep;
    }
    p->kcols = std::max(k_max, p->keep);
    p->onesided = 0;
    if (opts && opts->reorth != 0) {
        if (opts->reorth != 1 || (opts->restart_keep > 0)) {
            delete p;
            return SSA_EINVAL;
        }
        p->onesided = 1;
    }
    long long Mp;
    int M1, M2;
    if (!choose_fft(N, Mp, M1, M2)) {
        delete p;
        return SSA_EINVAL;
    }
    if (opts && opts->fft_mp > 0) {  // a longer transform: any M >= N gives the exact correlation
        const long long mp = opts->fft_mp;
        const int m1 = mp >= Mp && mp <= (long long)kMaxFactor * kMaxFactor ? balanced_m1(mp) : 0;
        if (m1 == 0) {
            delete p;
            return SSA_EINVAL;
        }
        Mp = mp;
        M1 = m1;
        M2 = (int)(mp / m1);
    }
    if (opts && opts->fft_m1 > 0) {  // schedule override: M1 must split M' into factors <= kMaxFactor
        const long long m1 = opts->fft_m1;
        if (Mp % m1 != 0 || m1 > kMaxFactor || Mp / m1 > kMaxFactor) {
            delete p;
            return SSA_EINVAL;
        }
        M1 = (int)m1;
        M2 = (int)(Mp / m1);
    }
    int cb = default_cb(M1, M2);
    if (opts && opts->fft_cb > 0) {
        // passes 1 and 3 hold CB columns of M1 points: at most 32 per thread of 256
        if (opts->fft_cb > 64 || (long long)opts->fft_cb * M1 > 8192) {
            delete p;
            return SSA_EINVAL;
        }
        cb = opts->fft_cb;
    }
    fill_geom(Mp, M1, M2, cb, p->g);
    const ConvGeom& gg = p->g;
    p->nblk = (gg.M2 + gg.CB - 1) / gg.CB;
    const int unfused = opts ? opts->unfused : 0;
    p->fused = (!is2d && p->keep == 0 && p->Ki <= kFusedMaxRows && unfused != 1) ? 1 : 0;
    // the fold: every pass-1 workgroup reads all partial sums, (ncols + 1) x nblk doubles
    p->fold = (p->fused && unfused == 0 && p->nblk <= kFoldMaxChunks) ? 1 : 0;
    if (p->fused) {
        // U-side vectors are outputs y[Ki-1+i] of X v, V-side ones y[Li-1+i] of X^T u
        p->layU = make_seglay(gg, p->Ki - 1, p->Li);
        p->layV = make_seglay(gg, p->Li - 1, p->Ki);
        p->ldU = (long long)align_up((size_t)p->layU.len, 64);
        p->ldV = (long long)align_up((size_t)p->layV.len, 64);
    } else {
        p->ldU = (long long)align_up((size_t)p->Li, 64);
        p->ldV = (long long)align_up((size_t)p->Ki, 64);
    }
    p->nchunks_max = (int)((std::max(p->ldU, p->ldV) + kProjRows - 1) / kProjRows);
    p->pstride = std::max(p->nchunks_max, p->fused ? p->nblk : 0);
    layout(p);
    p->work.resize(bidiag_work_doubles(d_max) + 16);
    *workspace_bytes = p->ws_bytes;
    *out = p;
    return SSA_OK;
}

int ssa_embed_plan(long long N, long long L, int k_max, const ssa_opts* opts, size_t* workspace_bytes,
                   ssa_plan* out) {
    if (!out || !workspace_bytes) return SSA_EINVAL;
    *out = nullptr;
    if (N <= 2 || L <= 1 || L >= N) return SSA_EINVAL;
    return plan_create(N, L, N - L + 1, 0, 0, 0, 0, 0, k_max, opts, workspace_bytes, out);
}

int ssa_embed_plan_2d(long long Nx, long long Ny, long long Lx, long long Ly, int k_max, const ssa_opts* opts,
                      size_t* workspace_bytes, ssa_plan* out) {
    if (!out || !workspace_bytes) return SSA_EINVAL;
    *out = nullptr;
    if (Nx < 1 || Ny < 1 || Lx < 1 || Ly < 1 || Lx > Nx || Ly > Ny) return SSA_EINVAL;
    if (Ny > (1LL << 30) || Nx > (1LL << 40) / Ny) return SSA_EINVAL;
    const long long L = Lx * Ly, K = (Nx - Lx + 1) * (Ny - Ly + 1);
    if (L < 2 || K < 2) return SSA_EINVAL;
    return plan_create(Nx * Ny, L, K, 1, Nx, Ny, Lx, Ly, k_max, opts, workspace_bytes, out);
}

int ssa_plan_bind(ssa_plan p, void* workspace_dev, size_t bytes, void* hip_stream) {
    if (!p || !workspace_dev) return SSA_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256) return SSA_EINVAL;
    if (bytes < p->ws_bytes) return SSA_ENOMEM;
    if (kernel_attributes_once() != hipSuccess) return SSA_EDEVICE;
    if (!p->h_scal) {
        ssa::PlanHost h;
        const int rc = ssa::host_alloc(h, host_scal_doubles(p->d_max, p->kcols, p->k_max), 2 * (size_t)p->nrec,
                                       p->grp_ints);
        if (rc != SSA_OK) {
            ssa::host_free(h);
            return rc;
        }
        use_host(p, h);
    }
    p->ws = static_cast<char*>(workspace_dev);
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->bound = 1;
    p->embedded = 0;
    const ConvGeom g = bound_geom(p);
    SSA_TRY(launch_tables(g, const_cast<float2*>(g.tw1), const_cast<float2*>(g.tw2), const_cast<float2*>(g.tw_lo),
                          const_cast<float2*>(g.tw_hi), p->stream));
    return SSA_OK;
}

int ssa_embed(ssa_plan p, const double* series_dev) {
    if (!p || !series_dev) return SSA_EINVAL;
    if (!p->bound) return SSA_ENOMEM;
    return do_embed(p, series_dev);
}

int ssa_matvec(ssa_plan p, int transpose, const float* x_dev, float* y_dev) {
    if (!p || !x_dev || !y_dev) return SSA_EINVAL;
    if (!p->bound) return SSA_ENOMEM;
    if (!p->embedded) return SSA_ESTATE;
    // X x: x has K entries; X^T x: x has L entries (user's L, K; side 0 is the shorter one)
    const int side = transpose ? (p->transposed ? 1 : 0) : (p->transposed ? 0 : 1);
    return convolve(p, bound_geom(p), x_dev, side, y_dev, nullptr, nullptr);
}

int ssa_truncated_svd(ssa_plan p, const double* series_dev, long long N, long long L, int k, double* sigma_dev,
                      float* U_dev, float* V_dev, ssa_info* info) {
    if (!p || !series_dev || !sigma_dev || !U_dev || !V_dev) return SSA_EINVAL;
    if (k < 1 || k > p->k_max) return SSA_EINVAL;
    if (N != p->N || L != p->L) return SSA_EMISMATCH;
    if (!p->bound) return SSA_ENOMEM;
    // Without thick restart the stopping test and the Ritz coefficients run on the
    // device and the host reads back only the test's record; the restarted solver
    // (below) assembles its projected matrix on the host.
    if (p->keep == 0) {
        int rc = ssa::run_begin(p, series_dev, k);
        while (rc == SSA_OK && !p->run.stopped) rc = ssa::run_advance(p, 1 << 30);
        if (rc != SSA_OK) {
            p->run.active = 0;
            p->stop_dev = nullptr;
            return rc;
        }
        return ssa::run_finish(p, sigma_dev, U_dev, V_dev, info);
    }
    int rc = do_embed(p, series_dev, true);
    if (rc != SSA_OK) return rc;
    const ConvGeom g = bound_geom(p);
    hipStream_t s = p->stream;
    const long long Li = p->Li, Ki = p->Ki;
    float* U = at<float>(p, p->o_U);
    float* V = at<float>(p, p->o_V);
    float* r = at<float>(p, p->o_r);
    double* alpha = at<double>(p, p->o_alpha);
    double* beta = at<double>(p, p->o_beta);
    SSA_TRY(launch_fill_zero(alpha, p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(beta, p->d_max + 3, s));
    SSA_TRY(launch_fill_zero(at<double>(p, p->o_state), 8, s));

    rc = start_vector(p);
    if (rc != SSA_OK) return rc;

    const int d_cap = (int)std::min<long long>(p->d_max, std::min(Li, Ki));
    const size_t abn = (size_t)(p->d_max + 3);
    double* h_ab[2] = {p->h_scal, p->h_scal + 2 * abn};  // alpha | beta, double-buffered
    double* h_P = p->h_scal + 4 * abn;
    double* h_Q = h_P + (size_t)(p->d_max + 1) * p->kcols;
    double* h_sig = h_Q + (size_t)p->d_max * p->kcols;
    std::vector<double> w(k), wprev(k), res(k);
    bool have_prev = false, converged = false;
    int d = 0, steps_run = 0;
    const double* fin = nullptr;
    // Stopping test on B_jj (its residual bound needs alpha_{jj+1}).  The test
    // of one check point runs on the host while the GPU works through the
    // steps enqueued after it, so the GPU never waits for the host; if it
    // stops there, the speculative steps beyond jj are discarded.
    auto evaluate = [&](int jj, const double* ab) -> bool {
        bidiag_ritz_values(ab, ab + abn, jj, k, w.data(), res.data(), p->work.data());
        bool ok = have_prev;
        for (int i = 0; i < k && ok; ++i) {
            const double scale = std::max(w[i], kResidFloor * w[0]);
            if (res[i] > p->tol * scale) ok = false;
            if (std::fabs(w[i] - wprev[i]) > 10.0 * p->tol * scale) ok = false;
        }
        if (jj >= std::min(Li, Ki)) ok = true;  // Krylov space exhausted: B is exact
        wprev = w;
        have_prev = true;
        if (ok || jj >= d_cap) {
            converged = ok;
            d = jj;
            fin = ab;
            return true;
        }
        return false;
    };
    int pend_jj = -1, pend_buf = 0, cur_buf = 0;
    for (int j = 1;; ++j) {
        rc = half_step(p, g, g, j, true);
        if (rc != SSA_OK) return rc;
        const int jj = j - 1;
        steps_run = jj;
        bool stop = false;
        if (jj >= k && (jj % p->check_every == 0 || jj >= d_cap)) {
            double* buf = h_ab[cur_buf];
            SSA_TRY(hipMemcpyAsync(buf, alpha, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
            SSA_TRY(hipMemcpyAsync(buf + abn, beta, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
            SSA_TRY(hipEventRecord(p->chk_ev[cur_buf], s));
            if (pend_jj >= 0) {
                SSA_TRY(hipEventSynchronize(p->chk_ev[pend_buf]));
                stop = evaluate(pend_jj, h_ab[pend_buf]);
            }
            if (!stop) {
                pend_jj = jj;
                pend_buf = cur_buf;
                cur_buf ^= 1;
                if (jj >= d_cap) {
                    SSA_TRY(hipEventSynchronize(p->chk_ev[pend_buf]));
                    stop = evaluate(jj, h_ab[pend_buf]);
                }
            }
        }
        if (stop) break;
        rc = half_step(p, g, g, j, false);
        if (rc != SSA_OK) return rc;
    }
    double* dP = at<double>(p, p->o_P);
    double* dQ = at<double>(p, p->o_Q);
    float* Uo = p->transposed ? V_dev : U_dev;  // internal U has length Li
    float* Vo = p->transposed ? U_dev : V_dev;
    const double* h_alpha = fin;
    const double* h_beta = fin + abn;
    int nu = d + 1, nc = d;  // the result is U_{nu} P (nu x k) and V_{nc} Q (nc x k)
    int cycles = 0;

    if (!converged && p->keep > 0 && d >= d_cap && d_cap < std::min(Li, Ki)) {
        // Thick restart (augmented Lanczos bidiagonalization, Sec. 3.3 on restarting).
        // With B = P Omega Q^T the SVD of the projected matrix and a the coefficient
        // of the newest V column, the m leading Ritz vectors satisfy
        //   X (V Q_m) = (U P_m) Omega_m,   X^T (U P_m) = (V Q_m) Omega_m + v_new rho^T,
        // rho_i = a P[last, i].  The bases restart as U' = U P_m, V' = [V Q_m, v_new]; the
        // projected matrix becomes diag(Omega_m) with rho as column m, and the recurrence
        // continues from v_new (its first product's component along U' is rho, which the
        // Gram-Schmidt step removes).  Every later step adds one bidiagonal pair, so each
        // cycle ends with a square nc x nc problem, solved densely on the host.
        const int m = p->keep;
        const size_t cap = (size_t)p->d_max + 1;
        const int kk = std::max(k, m);
        std::vector<double> Bm(cap * cap, 0.0), Bc, om(kk), PA, QA;
        for (int c = 0; c < d; ++c) {
            Bm[(size_t)c * cap + c] = h_alpha[c + 1];
            Bm[(size_t)(c + 1) * cap + c] = h_beta[c + 2];
        }
        double a_last = h_alpha[d + 1];
        float* rot = at<float>(p, p->o_rot);
        unsigned long long ctr = 2ULL * (unsigned long long)p->d_max + 8ULL;
        struct Fill { int row, col, from_beta, idx; };
        std::vector<Fill> fills;
        for (;;) {
            Bc.assign((size_t)nu * nc, 0.0);
            for (int r0 = 0; r0 < nu; ++r0)
                for (int c = 0; c < nc; ++c) Bc[(size_t)r0 * nc + c] = Bm[(size_t)r0 * cap + c];
            PA.assign((size_t)nu * kk, 0.0);
            QA.assign((size_t)nc * kk, 0.0);
            dense_ritz(Bc.data(), nu, nc, kk, om.data(), PA.data(), QA.data());
            if (cycles > 0) {  // cycle 0 is B_d, which the stopping test above has just rejected
                bool ok = have_prev;
                for (int i = 0; i < k; ++i) {
                    w[i] = om[i];
                    res[i] = std::fabs(a_last * PA[(size_t)(nu - 1) * kk + i]);
                    const double scale = std::max(w[i], kResidFloor * om[0]);
                    if (res[i] > p->tol * scale) ok = false;
                    if (std::fabs(w[i] - wprev[i]) > 10.0 * p->tol * scale) ok = false;
                }
                wprev = w;
                have_prev = true;
                if (ok || cycles >= kMaxCycles) {
                    converged = ok;
                    break;
                }
            }
            // rotate the bases: U' = U_{nu} P_m, V' = [V_{nc} Q_m, v_{nc+1}]
            for (int r0 = 0; r0 < nu; ++r0)
                for (int i = 0; i < m; ++i) h_P[(size_t)r0 * m + i] = PA[(size_t)r0 * kk + i];
            for (int r0 = 0; r0 < nc; ++r0)
                for (int i = 0; i < m; ++i) h_Q[(size_t)r0 * m + i] = QA[(size_t)r0 * kk + i];
            SSA_TRY(hipMemcpyAsync(dP, h_P, sizeof(double) * (size_t)nu * m, hipMemcpyHostToDevice, s));
            SSA_TRY(hipMemcpyAsync(dQ, h_Q, sizeof(double) * (size_t)nc * m, hipMemcpyHostToDevice, s));
            {
                ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Li * (nu + m));
                SSA_TRY(launch_ritz(U, p->ldU, nu, dP, m, rot, p->ldU, Li, s));
            }
            SSA_TRY(hipMemcpyAsync(U, rot, sizeof(float) * (size_t)m * p->ldU, hipMemcpyDeviceToDevice, s));
            {
                ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Ki * (nc + m));
                SSA_TRY(launch_ritz(V, p->ldV, nc, dQ, m, rot, p->ldV, Ki, s));
            }
            // nc >= m + 2 (keep + 2 <= d_max), so columns nc and m are distinct
            SSA_TRY(hipMemcpyAsync(V + (long long)m * p->ldV, V + (long long)nc * p->ldV, sizeof(float) * Ki,
                                   hipMemcpyDeviceToDevice, s));
            SSA_TRY(hipMemcpyAsync(V, rot, sizeof(float) * (size_t)m * p->ldV, hipMemcpyDeviceToDevice, s));
            std::fill(Bm.begin(), Bm.end(), 0.0);
            for (int i = 0; i < m; ++i) {
                Bm[(size_t)i * cap + i] = om[i];
                Bm[(size_t)i * cap + m] = a_last * PA[(size_t)(nu - 1) * kk + i];
            }
            ++cycles;
            // one cycle of the recurrence from v_{m+1}, until V holds d_cap + 1 columns
            nu = m;
            int nv = m + 1;
            fills.clear();
            bool first = true;
            while (nv - 1 < d_cap) {
                // p = X v_nv - alpha_nv u_nu (first step: the Gram-Schmidt step removes U' rho)
                rc = convolve(p, g, V + (long long)(nv - 1) * p->ldV, 1, r,
                              first ? nullptr : U + (long long)(nu - 1) * p->ldU, first ? nullptr : alpha + nv);
                if (rc != SSA_OK) return rc;
                rc = orthonormalize(p, U, p->ldU, nu, Li, beta + nu + 1, 1, ctr++);
                if (rc != SSA_OK) return rc;
                fills.push_back({nu, nv - 1, 1, nu + 1});
                ++nu;
                first = false;
                // r = X^T u_nu - beta_nu v_nv
                rc = convolve(p, g, U + (long long)(nu - 1) * p->ldU, 0, r, V + (long long)(nv - 1) * p->ldV,
                              beta + nu);
                if (rc != SSA_OK) return rc;
                rc = orthonormalize(p, V, p->ldV, nv, Ki, alpha + nv + 1, 1, ctr++);
                if (rc != SSA_OK) return rc;
                fills.push_back({nu - 1, nv, 0, nv + 1});
                ++nv;
                ++steps_run;
            }
            double* ha = h_ab[0];
            double* hb = h_ab[0] + abn;
            SSA_TRY(hipMemcpyAsync(ha, alpha, sizeof(double) * (size_t)(nv + 1), hipMemcpyDeviceToHost, s));
            SSA_TRY(hipMemcpyAsync(hb, beta, sizeof(double) * (size_t)(nu + 1), hipMemcpyDeviceToHost, s));
            SSA_TRY(hipStreamSynchronize(s));
            for (const Fill& f : fills) Bm[(size_t)f.row * cap + f.col] = (f.from_beta ? hb : ha)[f.idx];
            nc = nv - 1;
            a_last = ha[nv];
        }
        for (int i = 0; i < k; ++i) h_sig[i] = om[i];
        for (int r0 = 0; r0 < nu; ++r0)
            for (int i = 0; i < k; ++i) h_P[(size_t)r0 * k + i] = PA[(size_t)r0 * kk + i];
        for (int r0 = 0; r0 < nc; ++r0)
            for (int i = 0; i < k; ++i) h_Q[(size_t)r0 * k + i] = QA[(size_t)r0 * kk + i];
        d = steps_run;
    } else {
        // Ritz triples of B_d: sigma, U_{d+1} P, V_d Q
        bidiag_ritz_vectors(h_alpha, h_beta, d, k, h_sig, h_P, h_Q, p->work.data());
    }
    SSA_TRY(hipMemcpyAsync(dP, h_P, sizeof(double) * (size_t)nu * k, hipMemcpyHostToDevice, s));
    SSA_TRY(hipMemcpyAsync(dQ, h_Q, sizeof(double) * (size_t)nc * k, hipMemcpyHostToDevice, s));
    SSA_TRY(hipMemcpyAsync(sigma_dev, h_sig, sizeof(double) * k, hipMemcpyHostToDevice, s));
    {
        ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Li * (nu + k));
        if (p->fused)
            SSA_TRY(launch_ritz_seg(U, p->ldU, nu, dP, k, Uo, Li, p->layU, s));
        else
            SSA_TRY(launch_ritz(U, p->ldU, nu, dP, k, Uo, Li, Li, s));
    }
    {
        ProfScope ps(p, SSA_PROF_RITZ, 4.0 * (double)Ki * (nc + k));
        if (p->fused)
            SSA_TRY(launch_ritz_seg(V, p->ldV, nc, dQ, k, Vo, Ki, p->layV, s));
        else
            SSA_TRY(launch_ritz(V, p->ldV, nc, dQ, k, Vo, Ki, Ki, s));
    }
    double st[3] = {0, 0, 0};
    SSA_TRY(hipMemcpyAsync(h_sig + k, at<double>(p, p->o_state), sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    SSA_TRY(hipStreamSynchronize(s));
    std::memcpy(st, h_sig + k, sizeof(st));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->steps = d;
        info->converged = converged ? 1 : 0;
        info->restarts = (int)st[1];
        info->dgks_passes = (int)st[2];
        info->steps_run = steps_run;
        info->thick_restarts = cycles;
        info->half_step_launches = 6;
        for (int i = 0; i < k && i < 64; ++i) info->resid[i] = res[i];
    }
    const int status = !converged ? SSA_WARN_NOT_CONVERGED : st[1] > 0.0 ? SSA_WARN_BREAKDOWN : SSA_OK;
    if (info) info->status = status;
    return status;
}

int ssa_reconstruct(ssa_plan p, const double* sigma_dev, const float* U_dev, const float* V_dev, int k,
                    const int* group_offsets, const int* group_members, int m, float* out_dev) {
    if (!p || !sigma_dev || !U_dev || !V_dev || !group_offsets || !out_dev) return SSA_EINVAL;
    if (k < 1 || k > p->k_max || m < 1) return SSA_EINVAL;
    if (!p->bound) return SSA_ENOMEM;
    if (group_offsets[0] != 0) return SSA_EINVAL;
    std::vector<char> seen(k);
    for (int gi = 0; gi < m; ++gi) {
        const int b = group_offsets[gi], e = group_offsets[gi + 1];
        if (e < b || e - b > k) return SSA_EINVAL;
        if (e > b && !group_members) return SSA_EINVAL;
        std::fill(seen.begin(), seen.end(), 0);
        for (int t = b; t < e; ++t) {
            const int i = group_members[t];
            if (i < 0 || i >= k || seen[i]) return SSA_EINVAL;
            seen[i] = 1;
        }
    }
    const ConvGeom g = bound_geom(p);
    hipStream_t s = p->stream;
    const long long N = p->N, L = p->L, K = p->K;
    float2* T1 = at<float2>(p, p->o_rt1);
    float2* T2 = at<float2>(p, p->o_rt2);
    // spectra of every u_i and v_i (pass 1; pass 2 transforms the rows per group)
    P1In in{};
    in.U = U_dev;
    in.ldu = L;
    in.lenu = L;
    in.V = V_dev;
    in.ldv = K;
    in.lenv = K;
    in.nu = k;
    if (p->is2d) {  // U_i is Lx x Ly and V_i is Kx x Ky, row by row, scattered with row pitch Ny
        in.pitch = p->Ny;
        in.wu = (int)p->Ly;
        in.wv = (int)p->Ky;
        in.lenu = (p->Lx - 1) * p->Ny + p->Ly;
        in.lenv = (p->Kx - 1) * p->Ny + p->Ky;
    }
    {
        ProfScope ps(p, SSA_PROF_RECON1, 4.0 * (double)k * (L + K) + 16.0 * k * (double)g.Mp);
        SSA_TRY(launch_pass1(g, IN_VECS, in, 2 * k, T1, s));
    }
    int* dgrp = at<int>(p, p->o_grp);
    for (int g0 = 0; g0 < m; g0 += kMaxGroupBatch) {
        const int ng = std::min(kMaxGroupBatch, m - g0);
        // stage this batch's CSR (offsets rebased to 0) through pinned memory
        SSA_TRY(hipEventSynchronize(p->grp_done));
        const int base = group_offsets[g0];
        int nmem = 0;
        for (int gi = 0; gi <= ng; ++gi) p->h_grp[gi] = group_offsets[g0 + gi] - base;
        nmem = p->h_grp[ng];
        for (int t = 0; t < nmem; ++t) p->h_grp[ng + 1 + t] = group_members[base + t];
        SSA_TRY(hipMemcpyAsync(dgrp, p->h_grp, sizeof(int) * (size_t)(ng + 1 + nmem), hipMemcpyHostToDevice, s));
        SSA_TRY(hipEventRecord(p->grp_done, s));
        {
            ProfScope ps(p, SSA_PROF_RECON2, 16.0 * (double)g.Mp * nmem + 8.0 * (double)g.Mp * ng);
            SSA_TRY(launch_pass2_recon(g, T1, k, sigma_dev, dgrp, dgrp + ng + 1, 0, ng, T2, s));
        }
        P3Out o{};
        o.out = out_dev + (long long)g0 * N;
        o.N = N;
        o.L = L;
        o.K = K;
        o.ldo = N;
        if (p->is2d) {  // counts cnt_x(i) cnt_y(j)
            o.pitch = p->Ny;
            o.L = p->Ly;
            o.K = p->Ky;
            o.Nx = p->Nx;
            o.Lx = p->Lx;
            o.Kx = p->Kx;
        }
        {
            ProfScope ps(p, SSA_PROF_RECON3, (8.0 * (double)g.Mp + 4.0 * N) * ng);
            SSA_TRY(launch_pass3(g, OUT_HANKEL, T2, o, ng, s));
        }
        if (p->is2d) {
            ProfScope ps(p, SSA_PROF_RECON3, 4.0 * (double)N * ng);
            SSA_TRY(launch_recon_edges_2d(sigma_dev, U_dev, L, V_dev, K, dgrp, dgrp + ng + 1, ng, p->Nx, p->Ny, p->Lx,
                                          p->Ly, out_dev + (long long)g0 * N, N, s));
        } else {
            const long long lmin = std::min(L, K);
            const double ne = lmin <= kEdgeCnt ? (double)N : 2.0 * kEdgeCnt;
            ProfScope ps(p, SSA_PROF_RECON3, 4.0 * ne * ng);
            SSA_TRY(launch_recon_edges(sigma_dev, U_dev, L, V_dev, K, dgrp, dgrp + ng + 1, ng, N, L, K,
                                       out_dev + (long long)g0 * N, N, s));
        }
    }
    return SSA_OK;
}

int ssa_plan_describe(ssa_plan p, ssa_plan_desc* d) {
    if (!p || !d) return SSA_EINVAL;
    d->N = p->N;
    d->L = p->L;
    d->K = p->K;
    d->M = p->g.M;
    d->M1 = p->g.M1;
    d->M2 = p->g.M2;
    d->d_max = p->d_max;
    d->k_max = p->k_max;
    d->workspace_bytes = p->ws_bytes;
    d->cb = p->g.CB;
    return SSA_OK;
}

void ssa_plan_destroy(ssa_plan p) {
    if (!p) return;
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    if (p->lent) {  // the lender keeps its resources: only wait for this plan's work on them
        if (p->grp_done) (void)hipEventSynchronize(p->grp_done);
        if (p->chk_stream) (void)hipStreamSynchronize(p->chk_stream);
        delete p;
        return;
    }
    if (p->grp_done) {
        (void)hipEventSynchronize(p->grp_done);
        (void)hipEventDestroy(p->grp_done);
    }
    if (p->chk_stream) {
        (void)hipStreamSynchronize(p->chk_stream);
        (void)hipStreamDestroy(p->chk_stream);
    }
    if (p->ab_ev) (void)hipEventDestroy(p->ab_ev);
    if (p->run_ev) (void)hipEventDestroy(p->run_ev);
    for (hipEvent_t e : p->chk_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->h_scal) (void)hipHostFree(p->h_scal);
    if (p->h_flag) (void)hipHostFree(p->h_flag);
    if (p->h_rec) (void)hipHostFree(p->h_rec);
    if (p->h_grp) (void)hipHostFree(p->h_grp);
    delete p;
}

const char* ssa_status_str(int status) {
    switch (status) {
        case SSA_OK: return "ok";
        case SSA_WARN_NOT_CONVERGED: return "stopping rule not met before the Krylov dimension cap";
        case SSA_WARN_BREAKDOWN: return "converged after a breakdown (alpha or beta vanished; rank below k)";
        case SSA_EINVAL: return "invalid argument";
        case SSA_ENOMEM: return "workspace missing or too small";
        case SSA_ENONFINITE: return "series holds NaN or Inf";
        case SSA_EDEVICE: return "HIP runtime error";
        case SSA_EMISMATCH: return "N or L differ from the plan";
        case SSA_ESTATE: return "call order violated";
        default: return "unknown status";
    }
}

int ssa_profile_enable(ssa_plan p, unsigned class_mask) {
    if (!p) return SSA_EINVAL;
    if (p->stream || p->bound) (void)hipStreamSynchronize(p->stream);
    for (int c = 0; c < SSA_PROF_NCLASSES; ++c) {
        p->prof_pairs[c].clear();
        p->prof_bytes[c] = 0.0;
        p->prof_count[c] = 0;
        p->prof_seen[c] = 0;
    }
    p->ev_next = 0;
    p->prof_on = class_mask ? 1 : 0;
    p->prof_mask = class_mask;
    return SSA_OK;
}

int ssa_profile_read(ssa_plan p, int cls, long long* launches, double* ms, double* bytes) {
    if (!p || cls < 0 || cls >= SSA_PROF_NCLASSES) return SSA_EINVAL;
    if (p->bound && hipStreamSynchronize(p->stream) != hipSuccess) return SSA_EDEVICE;
    double total = 0.0;
    for (auto& pr : p->prof_pairs[cls]) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess) return SSA_EDEVICE;
        total += t;
    }
    // sampled timing: the mean of the timed launches stands for every launch of the class
    const size_t timed = p->prof_pairs[cls].size();
    if (timed) total *= (double)p->prof_count[cls] / (double)timed;
    if (launches) *launches = p->prof_count[cls];
    if (ms) *ms = (p->prof_on && (p->prof_mask >> cls & 1u)) ? total : -1.0;
    if (bytes) *bytes = p->prof_bytes[cls];
    return SSA_OK;
}

int ssa_profile_sample(ssa_plan p, int every) {
    if (!p || every < 1) return SSA_EINVAL;
    p->prof_every = every;
    return SSA_OK;
}

int ssa_bidiag_ritz(const double* alpha, const double* beta, int d, int k, double* omega, double* resid,
                    double* P, double* Q) {
    if (!alpha || !beta || !omega || d < 1 || k < 1) return SSA_EINVAL;
    std::vector<double> work(bidiag_work_doubles(d) + 16);
    if (resid) bidiag_ritz_values(alpha, beta, d, k, omega, resid, work.data());
    if (P && Q) bidiag_ritz_vectors(alpha, beta, d, k, omega, P, Q, work.data());
    return SSA_OK;
}

int ssa_dense_ritz(const double* A, int nr, int nc, int k, double* omega, double* P, double* Q) {
    if (!A || !omega || !P || !Q || nc < 1 || nr < nc || k < 1) return SSA_EINVAL;
    dense_ritz(A, nr, nc, k, omega, P, Q);
    return SSA_OK;
}

}  // extern "C"
