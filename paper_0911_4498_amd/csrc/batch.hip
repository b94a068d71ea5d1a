// batch.hip -- many independent series advanced in lockstep.
//
// Every launch has one workgroup per series of the batch (1024 threads for the
// kernels that hold an FFT in LDS, 512 for the others), and a series' result
// depends only on the series and its seed, never on what runs beside it.  Per Lanczos step the host enqueues
//   kb_conv, kb_cgs (j, side 0): r_j = X^T u_j - beta_j v_{j-1}, Gram-Schmidt
//                       against V, alpha_j, v_j         (Algorithm 1; Algorithm 3)
//   kb_check(j):        stopping test on B_{j-1}         (eqs. lbdiagm1/lbdiagm2)
//   kb_conv, kb_cgs (j, side 1): p_j = X v_j - alpha_j u_j, Gram-Schmidt
//                       against U, beta_{j+1}, u_{j+1}  (Algorithm 1; Algorithm 2)
// and after the last step kb_ritz (Ritz triples) and kb_hankel (rank-1
// Hankelization of every triple, Algorithm 4).  A series whose stopping rule
// held is skipped by every later launch.
//
// The product is the circular convolution of the zero-padded series with the
// reversed input vector (Sec. 4.2-4.3), done as a packed-real FFT of M' = M/2
// complex points entirely in one workgroup's LDS.  The Gram-Schmidt step runs
// in a second launch with small workgroups (several per CU, float4 rows from
// HBM): classical, FP64 sums of exact FP32 products, a second pass by the
// DGKS criterion and a seeded random restart on breakdown (Sec. 3.2.2).
//
// The stopping test works on T = B^T B (symmetric tridiagonal, T[c][c] =
// alpha_{c+1}^2 + beta_{c+2}^2, T[c][c+1] = alpha_{c+2} beta_{c+2}):
//  * its k largest eigenvalues by multisection on Sturm counts of the pivots
//    d_c(x) of T - x I;
//  * the last component of each eigenvector from the twisted factorization of
//    T - lambda I (products of pivot ratios, accurate for the tiny tails of
//    converged Ritz vectors);
//  * the residual bound alpha_{j+1} beta_{j+1} |q[n-1]| / omega (eq. lbdiagm2).
// The Ritz coefficients come from inverse iteration on T (one thread per
// triple) followed by modified Gram-Schmidt across the k vectors.
//
// All helpers are inlined into the kernels, so LDS is addressed directly.
#include <hip/hip_runtime.h>

#include "ssa_batch.h"
#include "tridiag_dev.h"

namespace ssa {
namespace batch {

#define SSA_INLINE __device__ __attribute__((always_inline)) inline

struct Lds {  // FFT-product, set-up and Hankelization kernels
    float2 buf[kMaxMp];
    float2 tw_hi[kTwTab];
    float2 tw_lo[kTwTab];
    double misc[kFftWaves];
};

// LDS of the stopping-test and Ritz kernels (no FFT buffer: several workgroups per CU)
struct SmallLds {
    double red[kWaves][kDmax + 2];
    double ab[2 * (kDmax + 3)];  // alpha | beta
    double tri[2 * (kDmax + 2)];
    double lo[kMaxK], hi[kMaxK], lam[kMaxK], qlast[kMaxK];
    double xs[kThreads];
    int cnt[kThreads];
    double misc[kWaves];
    double dmisc[8];
};

SSA_INLINE double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int W = kWaves, class S>
SSA_INLINE double block_sum(S* sh, double v, int tid) {
    v = wsum(v);
    __syncthreads();
    if ((tid & 63) == 0) sh->misc[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += sh->misc[w];
    __syncthreads();
    return s;
}

template <class S>
SSA_INLINE double block_max(S* sh, double v, int tid) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) sh->misc[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s = fmax(s, sh->misc[w]);
    __syncthreads();
    return s;
}

// Philox4x32-10 (Salmon et al., SC'11): counter (t, ctr), key = seed.
SSA_INLINE void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

// standard normal by Box-Muller from one Philox block
SSA_INLINE float gaussian(unsigned long long seed, unsigned long long ctr, long long t) {
    uint32_t c[4] = {(uint32_t)t, (uint32_t)((unsigned long long)t >> 32), (uint32_t)ctr, (uint32_t)(ctr >> 32)};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967296.0);
    const double u2 = (double)c[1] * (1.0 / 4294967296.0);
    return (float)(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
}

// real element m of the sequence packed in buf (w[2n] + i w[2n+1] at buf[n])
SSA_INLINE float getr(const float2* buf, long long m) {
    const float2 z = buf[m >> 1];
    return (m & 1) ? z.y : z.x;
}
SSA_INLINE void setr(float2* buf, long long m, float v) {
    if (m & 1)
        buf[m >> 1].y = v;
    else
        buf[m >> 1].x = v;
}

// Per-series constants of one launch.
struct Ser {
    long long N, Li, Ki, ldu, ldv;
    int k, dcap, Mp, tw_shift;
    unsigned long long seed;
    const FftStages* st;  // radix plan (in the series table)
    float4* AB;
    float2* tw;  // hi | lo tables, kTwTab each
    float* U;
    float* V;
    float* r;
    double* alpha;
    double* beta;
    double* state;
    double* P;
    double* Q;
    double* scr;
};

SSA_INLINE Ser load_series(const BatchArgs& a, int s) {
    const BSeries& b = a.tab[s];
    Ser r;
    r.N = b.N;
    r.Li = b.Li;
    r.Ki = b.Ki;
    r.ldu = b.ldu;
    r.ldv = b.ldv;
    r.k = b.k;
    r.dcap = b.dcap;
    r.Mp = b.Mp;
    r.tw_shift = b.tw_shift;
    r.seed = b.seed;
    r.st = &b.st;
    char* base = a.ws + b.reg;
    r.AB = reinterpret_cast<float4*>(base + b.o_ab);
    r.tw = reinterpret_cast<float2*>(base + b.o_tw);
    r.U = reinterpret_cast<float*>(base + b.o_u);
    r.V = reinterpret_cast<float*>(base + b.o_v);
    r.r = reinterpret_cast<float*>(base + b.o_r);
    r.alpha = reinterpret_cast<double*>(base + b.o_alpha);
    r.beta = reinterpret_cast<double*>(base + b.o_beta);
    r.state = reinterpret_cast<double*>(base + b.o_state);
    r.P = reinterpret_cast<double*>(base + b.o_p);
    r.Q = reinterpret_cast<double*>(base + b.o_q);
    r.scr = reinterpret_cast<double*>(base + b.o_scr);
    return r;
}

// M'-point complex FFT of buf in LDS (forward DIR = -1, inverse +1, no scaling)
template <int DIR>
SSA_INLINE void fft(Lds* sh, const Ser& q, int tid) {
    const TwoLevelTw tw{sh->tw_hi, sh->tw_lo, q.tw_shift};
    int p = 1;
    const int ns = q.st->nstages;
    for (int s = 0; s < ns; ++s) {
        const int R = q.st->radix[s];
        switch (R) {
            case 8: fft_stage<8, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
            case 4: fft_stage<4, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
            case 2: fft_stage<2, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
            case 3: fft_stage<3, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
            case 5: fft_stage<5, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
            default: fft_stage<7, DIR, kEpt>(sh->buf, q.Mp, 1, q.Mp, p, tw, tid, kFftThreads); break;
        }
        p *= R;
    }
}

SSA_INLINE void load_twiddles(Lds* sh, const Ser& q, int tid) {
    for (int t = tid; t < kTwTab; t += kFftThreads) {
        sh->tw_hi[t] = q.tw[t];
        sh->tw_lo[t] = q.tw[kTwTab + t];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// products (Algorithms 2 and 3)

// r = X x or X^T x (x: n_in entries in HBM) minus coef * prev, written to r_out
// (n_out entries); the product is y[n_in - 1 + t] of the circular convolution.
// Each phase issues all of a thread's global loads before it uses the first of them
// (at clamped, in-bounds positions; values past the data are replaced by zeros), so
// a phase waits for HBM once rather than once per loop iteration.  The twiddle tables
// are loaded here as well.
constexpr int kConvPts = kMaxMp / kFftThreads;              // input points per thread
constexpr int kConvPtBatch = 5;                              // input points whose loads fly together
constexpr int kConvPairs = (kMaxMp / 2) / kFftThreads + 1;  // bin pairs per thread
constexpr int kConvPairBatch = 3;                            // bin pairs whose operator loads fly together
constexpr int kConvOutBatch = 10;                            // outputs whose prev loads fly together
static_assert(kMaxMp % kFftThreads == 0 && kTwTab <= kFftThreads && 2 * kMaxMp < (1 << 30),
              "convolve's load layout");
SSA_INLINE void convolve(Lds* sh, const Ser& q, const float* x, long long n_in, long long n_out, const float* prev,
                         double coef, float* r_out, int tid) {
    float2* buf = sh->buf;
    const int wave0 = tid & ~63;  // (whole waves past the data skip their loads)
    const int nin = (int)n_in;    // <= 2 M'
    float2 th = make_float2(0.0f, 0.0f), tl = th;
    if (wave0 < kTwTab) {
        th = q.tw[min(tid, kTwTab - 1)];
        tl = q.tw[kTwTab + min(tid, kTwTab - 1)];
    }
    // the reversed input w[m] = x[n_in - 1 - m], packed w[2n] + i w[2n+1] at buf[n]
    for (int b = 0; b < kConvPts && wave0 + b * kFftThreads < q.Mp; b += kConvPtBatch) {
        float x0[kConvPtBatch], x1[kConvPtBatch];
#pragma unroll
        for (int i = 0; i < kConvPtBatch; ++i) {
            x0[i] = 0.0f;
            x1[i] = 0.0f;
            if (wave0 + (b + i) * kFftThreads >= q.Mp) continue;
            const int m0 = 2 * (tid + (b + i) * kFftThreads);
            x0[i] = x[max(nin - 1 - m0, 0)];
            x1[i] = x[max(nin - 2 - m0, 0)];
        }
        if (b == 0 && tid < kTwTab) {
            sh->tw_hi[tid] = th;
            sh->tw_lo[tid] = tl;
        }
#pragma unroll
        for (int i = 0; i < kConvPtBatch; ++i) {
            const int n = tid + (b + i) * kFftThreads, m0 = 2 * n;
            if (n < q.Mp) buf[n] = make_float2(m0 < nin ? x0[i] : 0.0f, m0 + 1 < nin ? x1[i] : 0.0f);
        }
    }
    __syncthreads();
    fft<-1>(sh, q, tid);
    // Q(k) = A(k) Z(k) + B(k) conj Z(M'-k), for the bin pair (k, M'-k) owned by one thread
    const int half = q.Mp / 2;
    for (int b = 0; b < kConvPairs && wave0 + b * kFftThreads <= half; b += kConvPairBatch) {
        float4 o0[kConvPairBatch], o1[kConvPairBatch];
#pragma unroll
        for (int i = 0; i < kConvPairBatch; ++i) {
            o0[i] = o1[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (wave0 + (b + i) * kFftThreads > half) continue;
            const int k = min(tid + (b + i) * kFftThreads, half);
            o0[i] = q.AB[k];
            o1[i] = q.AB[k == 0 ? 0 : q.Mp - k];
        }
#pragma unroll
        for (int i = 0; i < kConvPairBatch; ++i) {
            const int k = tid + (b + i) * kFftThreads;
            if (k > half) continue;
            const int kp = k == 0 ? 0 : q.Mp - k;
            const float2 z0 = buf[k], z1 = buf[kp];
            const float2 q0 = cadd(cmul(make_float2(o0[i].x, o0[i].y), z0), cmul(make_float2(o0[i].z, o0[i].w), cconj(z1)));
            const float2 q1 = cadd(cmul(make_float2(o1[i].x, o1[i].y), z1), cmul(make_float2(o1[i].z, o1[i].w), cconj(z0)));
            buf[k] = q0;
            if (kp != k) buf[kp] = q1;
        }
    }
    __syncthreads();
    fft<1>(sh, q, tid);
    const float cf = (float)coef;
    for (long long t0 = 0; t0 < n_out; t0 += (long long)kConvOutBatch * kFftThreads) {
        float pv[kConvOutBatch];
#pragma unroll
        for (int i = 0; i < kConvOutBatch; ++i) {
            pv[i] = 0.0f;
            if (!prev || t0 + wave0 + i * kFftThreads >= n_out) continue;
            pv[i] = prev[min(t0 + tid + i * kFftThreads, n_out - 1)];
        }
#pragma unroll
        for (int i = 0; i < kConvOutBatch; ++i) {
            const long long t = t0 + tid + i * kFftThreads;
            if (t >= n_out) continue;
            const float y = getr(buf, n_in - 1 + t);
            r_out[t] = prev ? y - cf * pv[i] : y;
        }
    }
}

// ---------------------------------------------------------------------------
// classical Gram-Schmidt (Sec. 3.2.2), one workgroup of kCgsThreads per series;
// r and the basis stream from HBM in float4 rows (ld is a multiple of 64)

struct CgsLds {
    double h[kDmax + 2];
    double red[kCgsWaves][kCgsCols + 1];
    double misc[kCgsWaves];
};

SSA_INLINE float4 rows4(const float* col, long long t, long long n) {
    float4 v = *reinterpret_cast<const float4*>(col + t);
    if (t + 3 >= n) {
        if (t + 1 >= n) v.y = 0.0f;
        if (t + 2 >= n) v.z = 0.0f;
        if (t + 3 >= n) v.w = 0.0f;
    }
    return v;
}

SSA_INLINE double dot4(float4 a, float4 b) {
    return (double)a.x * (double)b.x + (double)a.y * (double)b.y + (double)a.z * (double)b.z +
           (double)a.w * (double)b.w;
}

SSA_INLINE double cgs_sum(CgsLds* sh, double v, int tid) {
    v = wsum(v);
    __syncthreads();
    if ((tid & 63) == 0) sh->misc[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kCgsWaves; ++w) s += sh->misc[w];
    __syncthreads();
    return s;
}

// h[c] = <basis_c, r> for c < ncols and h[ncols] = |r|^2: FP64 sums of exact
// FP32 products in a fixed order, kCgsCols columns per pass over r.
SSA_INLINE void cgs_project(CgsLds* sh, const float* r, const float* basis, long long ld, int ncols, long long n,
                            int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    for (int c0 = 0; c0 <= ncols; c0 += kCgsCols) {
        double acc[kCgsCols + 1];
#pragma unroll
        for (int g = 0; g <= kCgsCols; ++g) acc[g] = 0.0;
        for (long long t = 4LL * tid; t < n; t += 4LL * kCgsThreads) {
            const float4 rv = rows4(r, t, n);
            if (c0 == 0) acc[kCgsCols] += dot4(rv, rv);
#pragma unroll
            for (int g = 0; g < kCgsCols; ++g)
                if (c0 + g < ncols) acc[g] += dot4(rows4(basis + (long long)(c0 + g) * ld, t, n), rv);
        }
#pragma unroll
        for (int g = 0; g <= kCgsCols; ++g) {
            const double v = wsum(acc[g]);
            if (lane == 0) sh->red[wave][g] = v;
        }
        __syncthreads();
        if (tid <= kCgsCols) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kCgsWaves; ++w) s += sh->red[w][tid];
            if (tid < kCgsCols && c0 + tid < ncols) sh->h[c0 + tid] = s;
            if (tid == kCgsCols && c0 == 0) sh->h[ncols] = s;
        }
        __syncthreads();
    }
}

// out = (r - basis h) * scale, FP64 accumulation (out may be r)
SSA_INLINE void cgs_update(const CgsLds* sh, const float* r, const float* basis, long long ld, int ncols,
                           long long n, double scale, float* out, int tid) {
    for (long long t = 4LL * tid; t < n; t += 4LL * kCgsThreads) {
        const float4 rv = rows4(r, t, n);
        double a0 = rv.x, a1 = rv.y, a2 = rv.z, a3 = rv.w;
#pragma unroll 8
        for (int c = 0; c < ncols; ++c) {
            const float4 b = rows4(basis + (long long)c * ld, t, n);
            const double hc = sh->h[c];
            a0 -= (double)b.x * hc;
            a1 -= (double)b.y * hc;
            a2 -= (double)b.z * hc;
            a3 -= (double)b.w * hc;
        }
        const float4 o = make_float4((float)(a0 * scale), (float)(a1 * scale), (float)(a2 * scale),
                                     (float)(a3 * scale));
        if (t + 3 < n) {
            *reinterpret_cast<float4*>(out + t) = o;
        } else {
            out[t] = o.x;
            if (t + 1 < n) out[t + 1] = o.y;
            if (t + 2 < n) out[t + 2] = o.z;
        }
    }
    __syncthreads();
}

SSA_INLINE double cgs_h2(CgsLds* sh, int ncols, int tid) {
    double hh = 0.0;
    for (int c = tid; c < ncols; c += kCgsThreads) hh += sh->h[c] * sh->h[c];
    return cgs_sum(sh, hh, tid);
}

// New basis column ncols from r: one Gram-Schmidt pass with
// |r_new|^2 = |r|^2 - |h|^2, a second pass if |r_new|^2 < |r|^2 / 2 (DGKS),
// a seeded random direction if the vector vanishes (|r_new| <= tol * max B).
// The random direction is made orthogonal to the first ncols_bd >= ncols columns:
// one-sided reorthogonalization projects the V side against no column (ncols = 0),
// yet a fresh direction must still be orthogonal to every earlier v (Sec. 3.2).
// Returns the B entry (0 after a restart); updates the series state.
SSA_INLINE double orthonormalize(CgsLds* sh, const Ser& q, float* r, float* basis, long long ld, int ncols,
                                 int ncols_bd, long long n, unsigned long long ctr, int tid, int out_col) {
    const double bnorm = q.state[kStBnorm];
    cgs_project(sh, r, basis, ld, ncols, n, tid);
    double coef = 0.0, scale = 0.0;
    int event = 0;  // 1: DGKS pass, 2: restart
    if (ncols >= n) {  // the basis already spans the space
        for (int c = tid; c < ncols; c += kCgsThreads) sh->h[c] = 0.0;
        __syncthreads();
    } else {
        const double hh = cgs_h2(sh, ncols, tid);
        const double rr = sh->h[ncols];
        double a2 = rr - hh;
        const double thr = kBreakdownTol * bnorm;
        if (a2 >= 0.5 * rr && sqrt(a2) > thr) {
            coef = sqrt(a2);
            scale = 1.0 / coef;
        } else {
            cgs_update(sh, r, basis, ld, ncols, n, 1.0, r, tid);
            cgs_project(sh, r, basis, ld, ncols, n, tid);
            const double hh2 = cgs_h2(sh, ncols, tid);
            a2 = sh->h[ncols] - hh2;
            if (a2 > 0.0 && sqrt(a2) > thr) {
                coef = sqrt(a2);
                scale = 1.0 / coef;
                event = 1;
            } else {
                for (long long t = tid; t < n; t += kCgsThreads) r[t] = gaussian(q.seed, ctr, t);
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    cgs_project(sh, r, basis, ld, ncols_bd, n, tid);
                    cgs_update(sh, r, basis, ld, ncols_bd, n, 1.0, r, tid);
                }
                cgs_project(sh, r, basis, ld, 0, n, tid);
                const double r3 = sh->h[0];
                for (int c = tid; c < ncols_bd; c += kCgsThreads) sh->h[c] = 0.0;
                __syncthreads();
                scale = r3 > 0.0 ? 1.0 / sqrt(r3) : 0.0;
                event = 2;
            }
        }
    }
    cgs_update(sh, r, basis, ld, ncols, n, scale, basis + (long long)out_col * ld, tid);
    if (tid == 0) {
        if (coef > bnorm) q.state[kStBnorm] = coef;
        if (event == 1) q.state[kStDgks] += 1.0;
        if (event == 2) q.state[kStRestarts] += 1.0;
    }
    return coef;
}

// ---------------------------------------------------------------------------
// kernels

// Spectral operator of each series (Algorithm 2, steps 1-2; packed form
// Q(k) = A Z(k) + B conj Z(M'-k), the 1/M' of the inverse folded in), the
// twiddle tables, the cleared state, and u_1 = p_0 / |p_0| for a seeded
// Gaussian p_0 (Algorithm 1, first line).
__global__ __launch_bounds__(kFftThreads) void kb_init(BatchArgs a) {
    extern __shared__ char lds[];
    Lds* sh = reinterpret_cast<Lds*>(lds);
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    const BSeries& b = a.tab[s];
    // twiddles W(t) = e^{-2 pi i t / M'}: lo[t] = W(t), hi[t] = W(t << shift)
    const int S = 1 << q.tw_shift;
    for (int t = tid; t < kTwTab; t += kFftThreads) {
        double sn, cs;
        float2 lo = make_float2(1.0f, 0.0f), hi = make_float2(1.0f, 0.0f);
        if (t < S) {
            sincospi(-2.0 * (double)t / (double)q.Mp, &sn, &cs);
            lo = make_float2((float)cs, (float)sn);
        }
        if ((long long)t * S < q.Mp) {
            sincospi(-2.0 * (double)((long long)t * S) / (double)q.Mp, &sn, &cs);
            hi = make_float2((float)cs, (float)sn);
        }
        q.tw[t] = hi;
        q.tw[kTwTab + t] = lo;
        sh->tw_hi[t] = hi;
        sh->tw_lo[t] = lo;
    }
    for (int i = tid; i < kDmax + 3; i += kFftThreads) {
        if (i <= q.dcap + 2) {
            q.alpha[i] = 0.0;
            q.beta[i] = 0.0;
        }
    }
    for (int i = tid; i < kStDoubles; i += kFftThreads) q.state[i] = i == kStJ ? 1.0 : 0.0;
    if (tid == 0 && a.done_flags) a.done_flags[s] = 0;
    const double* f = b.f;
    float2* buf = sh->buf;
    for (int n = tid; n < q.Mp; n += kFftThreads) {
        const long long m0 = 2LL * n, m1 = m0 + 1;
        buf[n] = make_float2(m0 < q.N ? (float)f[m0] : 0.0f, m1 < q.N ? (float)f[m1] : 0.0f);
    }
    __syncthreads();
    fft<-1>(sh, q, tid);
    const double invMp = 1.0 / (double)q.Mp;
    const double M = 2.0 * q.Mp;
    for (int k = tid; k < q.Mp; k += kFftThreads) {
        const int kp = k == 0 ? 0 : q.Mp - k;
        const float2 z = buf[k], zp = buf[kp];
        const double er = 0.5 * ((double)z.x + (double)zp.x), ei = 0.5 * ((double)z.y - (double)zp.y);
        const double orr = 0.5 * ((double)z.y + (double)zp.y), oi = -0.5 * ((double)z.x - (double)zp.x);
        double sn, cs;
        sincospi(2.0 * (double)k / M, &sn, &cs);
        const double wor = cs * orr + sn * oi, woi = cs * oi - sn * orr;
        const double ar = (er - sn * wor) * invMp, ai = (ei - sn * woi) * invMp;
        const double br = -cs * woi * invMp, bi = cs * wor * invMp;
        q.AB[k] = make_float4((float)ar, (float)ai, (float)br, (float)bi);
    }
    __syncthreads();
    // start vector
    double ss = 0.0;
    for (long long t = tid; t < q.Li; t += kFftThreads) {
        const float g = gaussian(q.seed, 0, t);
        q.U[t] = g;
        ss += (double)g * (double)g;
    }
    ss = block_sum<kFftWaves>(sh, ss, tid);
    const double nrm = sqrt(ss);
    const float sc = (float)(1.0 / nrm);
    for (long long t = tid; t < q.Li; t += kFftThreads) q.U[t] *= sc;
    if (tid == 0) {
        q.beta[1] = nrm;
        q.state[kStBnorm] = nrm;
    }
}

// One half of Lanczos step j for every unfinished series, product part:
//   side 0: r = X^T u_j - beta_j v_{j-1};   side 1: r = X v_j - alpha_j u_j.
__global__ __launch_bounds__(kFftThreads) void kb_conv(BatchArgs a, int side) {
    extern __shared__ char lds[];
    Lds* sh = reinterpret_cast<Lds*>(lds);
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    const int j = (int)q.state[kStJ];
    if (q.state[kStDone] != 0.0 || j - 1 > q.dcap) return;
    if (side == 0)
        convolve(sh, q, q.U + (long long)(j - 1) * q.ldu, q.Li, q.Ki,
                 j >= 2 ? q.V + (long long)(j - 2) * q.ldv : nullptr, q.beta[j], q.r, tid);
    else
        convolve(sh, q, q.V + (long long)(j - 1) * q.ldv, q.Ki, q.Li, q.U + (long long)(j - 1) * q.ldu,
                 q.alpha[j], q.r, tid);
}

// Gram-Schmidt part: side 0: v_j and alpha_j;  side 1: u_{j+1} and beta_{j+1}.
// (six waves per SIMD: at most 80 VGPRs, no spills, three workgroups per CU)
__global__ __launch_bounds__(kCgsThreads, 6) void kb_cgs(BatchArgs a, int side) {
    extern __shared__ char lds[];
    CgsLds* sh = reinterpret_cast<CgsLds*>(lds);
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    const int j = (int)q.state[kStJ];
    if (q.state[kStDone] != 0.0 || j - 1 > q.dcap) return;
    if (side == 0) {
        // one-sided: V (length Ki >= Li) keeps only the three-term recurrence
        const double aj = orthonormalize(sh, q, q.r, q.V, q.ldv, a.onesided ? 0 : j - 1, j - 1, q.Ki, 2ULL * j, tid, j - 1);
        if (tid == 0) q.alpha[j] = aj;
    } else {
        const double bj = orthonormalize(sh, q, q.r, q.U, q.ldu, j, j, q.Li, 2ULL * j + 1, tid, j);
        if (tid == 0) {
            q.beta[j + 1] = bj;
            q.state[kStJ] = (double)(j + 1);  // the series' next Lanczos step
        }
    }
}

// The k largest eigenvalues of T_n by multisection (sh->lam); D, E2 in sh->tri,
// the pivot floor in sh->dmisc[0].
SSA_INLINE void tridiag_top(SmallLds* sh, int n, int k, int tid) {
    const double* al = sh->ab;
    const double* be = sh->ab + (kDmax + 3);
    double* D = sh->tri;
    double* E2 = sh->tri + kDmax + 2;
    for (int i = tid; i < n; i += kThreads) {
        const double x = al[i + 1], y = be[i + 2];
        D[i] = x * x + y * y;
        if (i + 1 < n) {
            const double e = al[i + 2] * be[i + 2];
            E2[i] = e * e;
        }
    }
    __syncthreads();
    double g = 0.0, e2max = 0.0;
    for (int i = tid; i < n; i += kThreads) {
        const double el = i > 0 ? sqrt(E2[i - 1]) : 0.0, er = i + 1 < n ? sqrt(E2[i]) : 0.0;
        g = fmax(g, D[i] + el + er);
        if (i + 1 < n) e2max = fmax(e2max, E2[i]);
    }
    const double gmax = block_max(sh, g, tid);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, block_max(sh, e2max, tid));
    for (int i = tid; i < k; i += kThreads) {
        sh->lo[i] = 0.0;
        sh->hi[i] = gmax * (1.0 + 1e-12) + 1e-300;
    }
    __syncthreads();
    multisection_top<kThreads>(D, E2, n, k, pivmin, sh->lo, sh->hi, sh->xs, sh->cnt, 14, tid);
    for (int i = tid; i < k; i += kThreads) sh->lam[i] = 0.5 * (sh->lo[i] + sh->hi[i]);
    if (tid == 0) sh->dmisc[0] = pivmin;
    __syncthreads();
}

// Stopping test of step j on B_{j-1} for the series whose check point it is:
// every residual bound <= tol * max(omega_i, 1e-5 omega_1) and the k Ritz
// values within 10 tol (relative) of the previous check's; or the Krylov cap.
__global__ __launch_bounds__(kThreads) void kb_check(BatchArgs a) {
    extern __shared__ char lds[];
    SmallLds* sh = reinterpret_cast<SmallLds*>(lds);
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    if (q.state[kStDone] != 0.0) return;
    const int j = (int)q.state[kStJ];
    const int jj = j - 1, k = q.k;
    if (!(jj >= k && (jj % a.check_every == 0 || jj >= q.dcap))) return;
    for (int i = tid; i <= jj + 1; i += kThreads) {
        sh->ab[i] = q.alpha[i];
        sh->ab[kDmax + 3 + i] = q.beta[i];
    }
    __syncthreads();
    tridiag_top(sh, jj, k, tid);
    if (tid < k) {
        double* dm = q.scr + (long long)tid * 2 * (q.dcap + 2);
        sh->qlast[tid] = twisted_qlast(sh->tri, sh->tri + kDmax + 2, jj, sh->lam[tid], sh->dmisc[0], dm,
                                       dm + (q.dcap + 2));
    }
    __syncthreads();
    if (tid == 0) {
        const double w0 = sqrt(fmax(sh->lam[0], 0.0));
        bool ok = q.state[kStHavePrev] != 0.0;
        const double ab = sh->ab[jj + 1] * sh->ab[kDmax + 3 + jj + 1];
        for (int i = 0; i < k; ++i) {
            const double w = sqrt(fmax(sh->lam[i], 0.0));
            const double res = w > 0.0 ? ab * sqrt(sh->qlast[i]) / w : 0.0;
            const double sc = fmax(w, kResidFloor * w0);
            if (res > a.tol * sc) ok = false;
            if (fabs(w - q.state[kStWprev + i]) > 10.0 * a.tol * sc) ok = false;
            q.state[kStWprev + i] = w;
            q.state[kStResid + i] = res;
            q.state[kStLam + i] = sh->lam[i];
        }
        q.state[kStHavePrev] = 1.0;
        const bool exhausted = jj >= q.Li;  // the Krylov space is exhausted: B is exact
        if (ok || exhausted || jj >= q.dcap) {
            q.state[kStDone] = 1.0;
            q.state[kStD] = (double)jj;
            q.state[kStConv] = (ok || exhausted) ? 1.0 : 0.0;
            if (a.ndone) atomicAdd(a.ndone, 1u);
            if (a.done_flags) a.done_flags[s] = 1;
        }
    }
}

// Column i of the (n x k, row-major) left coefficient matrix P made orthogonal to
// columns 0..i-1 by two Gram-Schmidt passes; returns its norm.
SSA_INLINE double left_orth(SmallLds* sh, double* P, int k, int n, int i, int tid) {
    for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < i; ++j) {
            double h = 0.0;
            for (int r = tid; r < n; r += kThreads) h += P[(long long)r * k + j] * P[(long long)r * k + i];
            h = block_sum(sh, h, tid);
            for (int r = tid; r < n; r += kThreads) P[(long long)r * k + i] -= h * P[(long long)r * k + j];
            __syncthreads();
        }
    double nrm = 0.0;
    for (int r = tid; r < n; r += kThreads) nrm += P[(long long)r * k + i] * P[(long long)r * k + i];
    return sqrt(block_sum(sh, nrm, tid));
}

// out[i*ldo + t] = sum_{c < ncols} basis[c][t] coef[c*k + i], i < k
SSA_INLINE void ritz_vectors(SmallLds* sh, const float* basis, long long ld, int ncols, const double* coef, int k,
                             float* out, long long ldo, long long n, int tid) {
    constexpr int T = 8;
    double* cs = &sh->red[0][0];  // ncols x T coefficients
    for (int i0 = 0; i0 < k; i0 += T) {
        for (int idx = tid; idx < ncols * T; idx += kThreads) {
            const int c = idx / T, i = idx % T;
            cs[idx] = i0 + i < k ? coef[(long long)c * k + i0 + i] : 0.0;
        }
        __syncthreads();
        for (long long t = tid; t < n; t += kThreads) {
            double acc[T];
#pragma unroll
            for (int i = 0; i < T; ++i) acc[i] = 0.0;
            for (int c = 0; c < ncols; ++c) {
                const double x = basis[(long long)c * ld + t];
#pragma unroll
                for (int i = 0; i < T; ++i) acc[i] += x * cs[c * T + i];
            }
#pragma unroll
            for (int i = 0; i < T; ++i)
                if (i0 + i < k) out[(long long)(i0 + i) * ldo + t] = (float)acc[i];
        }
        __syncthreads();
    }
}

// Ritz triples of B_d: Q (d x k) by inverse iteration on T at the eigenvalues
// of the last check plus modified Gram-Schmidt, P = B Q / |B Q|; then sigma,
// U_{d+1} P and V_d Q in the caller's layout, and the per-series report.
__global__ __launch_bounds__(kThreads) void kb_ritz(BatchArgs a) {
    extern __shared__ char lds[];
    SmallLds* sh = reinterpret_cast<SmallLds*>(lds);
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    const BSeries& b = a.tab[s];
    const int k = q.k;
    const int d = (int)q.state[kStD];
    for (int i = tid; i <= d + 1; i += kThreads) {
        sh->ab[i] = q.alpha[i];
        sh->ab[kDmax + 3 + i] = q.beta[i];
    }
    for (int i = tid; i < k; i += kThreads) sh->lam[i] = q.state[kStLam + i];
    __syncthreads();
    const double* al = sh->ab;
    const double* be = sh->ab + (kDmax + 3);
    double* D = sh->tri;
    double* E = sh->tri + kDmax + 2;  // off-diagonal (not squared)
    for (int i = tid; i < d; i += kThreads) {
        const double x = al[i + 1], y = be[i + 2];
        D[i] = x * x + y * y;
        if (i + 1 < d) E[i] = al[i + 2] * be[i + 2];
    }
    __syncthreads();
    double g = 0.0;
    for (int i = tid; i < d; i += kThreads) g = fmax(g, fabs(D[i]) + 2.0 * (i + 1 < d ? fabs(E[i]) : 0.0));
    const double tnorm = block_max(sh, g, tid);
    const long long stride = q.dcap + 2;
    if (tid < k && tid < d) {
        const int i = tid;
        double* x = q.scr + (long long)i * 5 * stride;
        double* wa = x + stride;
        double* wb = wa + stride;
        double* wc = wb + stride;
        double* wu = wc + stride;
        for (int t = 0; t < d; ++t) x[t] = 1.0 + 0.5 * sin(0.7 * (t + 1) + 1.3 * (i + 1));
        for (int it = 0; it < 4; ++it) {
            shifted_solve(D, E, d, sh->lam[i], tnorm, x, wa, wb, wc, wu);
            double nrm = 0.0;
            for (int t = 0; t < d; ++t) nrm += x[t] * x[t];
            nrm = sqrt(nrm);
            if (!(nrm > 0.0) || !isfinite(nrm)) {
                for (int t = 0; t < d; ++t) x[t] = t == i ? 1.0 : 0.0;
                nrm = 1.0;
            }
            for (int t = 0; t < d; ++t) x[t] /= nrm;
        }
    }
    __syncthreads();
    double bm = 0.0;
    for (int i = tid; i < d; i += kThreads) bm = fmax(bm, fmax(fabs(al[i + 1]), fabs(be[i + 2])));
    const double bmax = block_max(sh, bm, tid);
    const int kk = k < d ? k : d;
    for (int i = 0; i < kk; ++i) {
        double* xi = q.scr + (long long)i * 5 * stride;
        for (int p = 0; p < i; ++p) {
            const double* xp = q.scr + (long long)p * 5 * stride;
            double dt = 0.0;
            for (int t = tid; t < d; t += kThreads) dt += xp[t] * xi[t];
            dt = block_sum(sh, dt, tid);
            for (int t = tid; t < d; t += kThreads) xi[t] -= dt * xp[t];
            __syncthreads();
        }
        double nrm = 0.0;
        for (int t = tid; t < d; t += kThreads) nrm += xi[t] * xi[t];
        nrm = sqrt(block_sum(sh, nrm, tid));
        for (int t = tid; t < d; t += kThreads) {
            xi[t] = nrm > 0.0 ? xi[t] / nrm : 0.0;
            q.Q[(long long)t * k + i] = xi[t];
        }
        __syncthreads();
        // p = B q, kept orthogonal to the earlier left vectors (two passes); when it
        // vanishes (omega_i = 0, a series of rank below k) a unit vector orthogonal to
        // them completes the SVD of B instead
        for (int r = tid; r <= d; r += kThreads) {
            double v = 0.0;
            if (r < d) v += al[r + 1] * xi[r];
            if (r >= 1) v += be[r + 1] * xi[r - 1];
            q.P[(long long)r * k + i] = v;
        }
        __syncthreads();
        double pn = left_orth(sh, q.P, k, d + 1, i, tid);
        for (int c = d; !(pn > 1e-12 * bmax) && c >= 0; --c) {
            for (int r = tid; r <= d; r += kThreads) q.P[(long long)r * k + i] = r == c ? 1.0 : 0.0;
            __syncthreads();
            pn = left_orth(sh, q.P, k, d + 1, i, tid);
            if (pn < 0.5) pn = 0.0;
        }
        for (int r = tid; r <= d; r += kThreads) q.P[(long long)r * k + i] = pn > 0.0 ? q.P[(long long)r * k + i] / pn : 0.0;
        __syncthreads();
    }
    for (int i = kk; i < k; ++i) {
        for (int t = tid; t < d; t += kThreads) q.Q[(long long)t * k + i] = 0.0;
        for (int r = tid; r <= d; r += kThreads) q.P[(long long)r * k + i] = 0.0;
    }
    __syncthreads();
    float* Uo = b.U;
    float* Vo = b.V;
    float* Ui = b.transposed ? Vo : Uo;  // the internal U has Li entries
    float* Vi = b.transposed ? Uo : Vo;
    ritz_vectors(sh, q.U, q.ldu, d + 1, q.P, k, Ui, q.Li, q.Li, tid);
    ritz_vectors(sh, q.V, q.ldv, d, q.Q, k, Vi, q.Ki, q.Ki, tid);
    for (int i = tid; i < k; i += kThreads) b.sigma[i] = sqrt(fmax(sh->lam[i], 0.0));
    if (tid == 0 && b.info) {
        int* inf = b.info;
        inf[0] = d;
        inf[1] = (int)q.state[kStConv];
        inf[2] = (int)q.state[kStRestarts];
        inf[3] = (int)q.state[kStDgks];
    }
}

// Elementary series of every triple (Algorithm 4): g = sigma (u * v) / cnt,
// the linear convolution by a packed-real FFT; the spectrum of u waits in the
// region's scratch while v is transformed.  Entries whose antidiagonal has at
// most kEdge terms are summed directly (FP64 sums of exact FP32 products, in
// ascending order of the u index).  When L and K both exceed kEdge those entries
// sit at the two ends of the series and read only the first and last kEdge
// entries of u and v, which are staged in LDS once the product is done.
struct HankelLds {
    Lds fft;
    float edge[4][kEdge];  // u head, u tail, v head, v tail
};

__global__ __launch_bounds__(kFftThreads) void kb_hankel(BatchArgs a) {
    extern __shared__ char lds[];
    HankelLds* hl = reinterpret_cast<HankelLds*>(lds);
    Lds* sh = &hl->fft;
    const int tid = threadIdx.x, s = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
    const Ser q = load_series(a, s);
    const BSeries& b = a.tab[s];
    if (!b.recon) return;
    load_twiddles(sh, q, tid);
    float2* buf = sh->buf;
    float2* zu = reinterpret_cast<float2*>(q.scr);
    const long long N = q.N, L = b.L, K = N - b.L + 1;
    const int Mp = q.Mp;
    const double M = 2.0 * Mp;
    const bool staged = L > kEdge && K > kEdge;  // (uniform)
    for (int i = 0; i < q.k; ++i) {
        const double sigma = b.sigma[i];
        const float* u = b.U + (long long)i * L;
        const float* v = b.V + (long long)i * K;
        float* out = b.recon + (long long)i * N;
        for (int n = tid; n < Mp; n += kFftThreads) {
            const long long m0 = 2LL * n, m1 = m0 + 1;
            buf[n] = make_float2(m0 < L ? u[m0] : 0.0f, m1 < L ? u[m1] : 0.0f);
        }
        __syncthreads();
        fft<-1>(sh, q, tid);
        for (int n = tid; n < Mp; n += kFftThreads) zu[n] = buf[n];
        __syncthreads();
        for (int n = tid; n < Mp; n += kFftThreads) {
            const long long m0 = 2LL * n, m1 = m0 + 1;
            buf[n] = make_float2(m0 < K ? v[m0] : 0.0f, m1 < K ? v[m1] : 0.0f);
        }
        __syncthreads();
        fft<-1>(sh, q, tid);
        const double sc = sigma / (double)Mp;
        for (int k = tid; k <= Mp / 2; k += kFftThreads) {
            const int kp = k == 0 ? 0 : Mp - k;
            const float2 zu0 = zu[k], zu1 = zu[kp];
            const float2 zv0 = buf[k], zv1 = buf[kp];
            for (int side = 0; side < 2; ++side) {
                if (side == 1 && kp == k) break;
                const float2 x = side == 0 ? zu0 : zu1, xp = side == 0 ? zu1 : zu0;
                const float2 y = side == 0 ? zv0 : zv1, yp = side == 0 ? zv1 : zv0;
                const int kk = side == 0 ? k : kp;
                double sn, cs;
                sincospi(2.0 * (double)kk / M, &sn, &cs);
                const double wr = cs, wi = -sn;
                // E/O split of each spectrum, then the full spectra at kk and kk + M'
                const double uer = 0.5 * ((double)x.x + (double)xp.x), uei = 0.5 * ((double)x.y - (double)xp.y);
                const double uor = 0.5 * ((double)x.y + (double)xp.y), uoi = -0.5 * ((double)x.x - (double)xp.x);
                const double ver = 0.5 * ((double)y.x + (double)yp.x), vei = 0.5 * ((double)y.y - (double)yp.y);
                const double vor = 0.5 * ((double)y.y + (double)yp.y), voi = -0.5 * ((double)y.x - (double)yp.x);
                const double uwr = wr * uor - wi * uoi, uwi = wr * uoi + wi * uor;
                const double vwr = wr * vor - wi * voi, vwi = wr * voi + wi * vor;
                const double uar = uer + uwr, uai = uei + uwi, ubr = uer - uwr, ubi = uei - uwi;
                const double var_ = ver + vwr, vai = vei + vwi, vbr = ver - vwr, vbi = vei - vwi;
                const double gar = uar * var_ - uai * vai, gai = uar * vai + uai * var_;
                const double gbr = ubr * vbr - ubi * vbi, gbi = ubr * vbi + ubi * vbr;
                const double dr = gar - gbr, di = gai - gbi;
                const double tr = dr * wr + di * wi, ti = di * wr - dr * wi;
                const double qr = 0.5 * (gar + gbr) - 0.5 * ti, qi = 0.5 * (gai + gbi) + 0.5 * tr;
                buf[kk] = make_float2((float)(qr * sc), (float)(qi * sc));
            }
        }
        __syncthreads();
        fft<1>(sh, q, tid);
        if (staged) {
            float ev[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if ((tid & ~63) < kEdge) {  // (whole waves past the edges skip the loads)
                const int t = min(tid, kEdge - 1);
                ev[0] = u[t];
                ev[1] = u[L - kEdge + t];
                ev[2] = v[t];
                ev[3] = v[K - kEdge + t];
            }
            if (tid < kEdge) {
#pragma unroll
                for (int e = 0; e < 4; ++e) hl->edge[e][tid] = ev[e];
            }
            __syncthreads();
        }
        for (long long m = tid; m < N; m += kFftThreads) {
            long long cnt = m + 1;
            if (L < cnt) cnt = L;
            if (K < cnt) cnt = K;
            if (N - m < cnt) cnt = N - m;
            if (cnt <= kEdge) {
                double acc = 0.0;
                if (staged && m < kEdge) {  // u[0 .. m] against v[m .. 0]
                    const int mm = (int)m;
                    for (int t = 0; t <= mm; ++t) acc += (double)hl->edge[0][t] * (double)hl->edge[2][mm - t];
                } else if (staged) {  // u[m - K + 1 .. L - 1] (the last cnt of u) against v[K - 1 .. m - L + 1]
                    // u[L - kEdge + j] = tail[j]; its partner v[m - L + kEdge - j] = vtail[2 kEdge - cnt - 1 - j]
                    const int c = (int)cnt;
                    for (int j = kEdge - c; j < kEdge; ++j)
                        acc += (double)hl->edge[1][j] * (double)hl->edge[3][2 * kEdge - c - 1 - j];
                } else {
                    const long long a0 = m - K + 1 > 0 ? m - K + 1 : 0, a1 = m < L - 1 ? m : L - 1;
                    for (long long t = a0; t <= a1; ++t) acc += (double)u[t] * (double)v[m - t];
                }
                out[m] = (float)(sigma * acc / (double)cnt);
            } else {
                out[m] = getr(buf, m) / (float)cnt;
            }
        }
        __syncthreads();
    }
}

#undef SSA_INLINE

}  // namespace batch

static hipError_t allow_lds(const void* f, size_t bytes = sizeof(batch::Lds)) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static hipError_t batch_attributes() {
    static hipError_t err = [] {
        hipError_t e = hipSuccess;
        for (const void* f : {reinterpret_cast<const void*>(batch::kb_init), reinterpret_cast<const void*>(batch::kb_conv),
                              reinterpret_cast<const void*>(batch::kb_check), reinterpret_cast<const void*>(batch::kb_ritz)}) {
            const hipError_t e2 = allow_lds(f);
            if (e2 != hipSuccess) e = e2;
        }
        const hipError_t e3 = allow_lds(reinterpret_cast<const void*>(batch::kb_hankel), sizeof(batch::HankelLds));
        return e != hipSuccess ? e : e3;
    }();
    return err;
}

hipError_t launch_batch_init(const BatchArgs& a, hipStream_t s) {
    const hipError_t e = batch_attributes();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch::kb_init, dim3(a.nseries), dim3(batch::kFftThreads), sizeof(batch::Lds), s, a);
    return hipGetLastError();
}

hipError_t launch_batch_conv(const BatchArgs& a, int side, hipStream_t s) {
    hipLaunchKernelGGL(batch::kb_conv, dim3(a.nseries), dim3(batch::kFftThreads), sizeof(batch::Lds), s, a, side);
    return hipGetLastError();
}

hipError_t launch_batch_cgs(const BatchArgs& a, int side, hipStream_t s) {
    hipLaunchKernelGGL(batch::kb_cgs, dim3(a.nseries), dim3(batch::kCgsThreads), sizeof(batch::CgsLds), s, a,
                       side);
    return hipGetLastError();
}

hipError_t launch_batch_check(const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(batch::kb_check, dim3(a.nseries), dim3(batch::kThreads), sizeof(batch::SmallLds), s, a);
    return hipGetLastError();
}

hipError_t launch_batch_ritz(const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(batch::kb_ritz, dim3(a.nseries), dim3(batch::kThreads), sizeof(batch::SmallLds), s, a);
    return hipGetLastError();
}

hipError_t launch_batch_hankel(const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(batch::kb_hankel, dim3(a.nseries), dim3(batch::kFftThreads), sizeof(batch::HankelLds), s, a);
    return hipGetLastError();
}

size_t batch_lds_bytes() { return sizeof(batch::Lds); }

}  // namespace ssa
