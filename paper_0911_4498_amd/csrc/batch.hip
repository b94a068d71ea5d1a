// batch.hip -- many independent series in one persistent launch.
//
// Every workgroup (1024 threads, one per CU) repeatedly takes the next series
// from a work counter and runs the whole hot path for it: the spectrum of the
// series (Algorithm 2, steps 1-2), Golub-Kahan-Lanczos bidiagonalization with
// full classical Gram-Schmidt reorthogonalization (Algorithm 1, Sec. 3.2.2)
// whose products X v / X^T u are FFT convolutions done entirely in LDS
// (Algorithms 2/3), the stopping test on B_j (eqs. lbdiagm1/lbdiagm2), the Ritz
// triples, and the rank-1 Hankelization of every triple (Algorithm 4).  A
// series' result depends only on the series, its index and the seed -- never
// on which workgroup ran it or what ran beside it -- and no workgroup waits
// for another (the only shared state is the work counter).
//
// Sizes: the FFT of a series has M' = M/2 <= kMaxMp complex points (M >= N the
// smallest even length with a 7-smooth half), held in LDS with two small
// twiddle tables.  The Lanczos bases of the series live in the workgroup's
// slot of HBM.
//
// The stopping test and the Ritz vectors use T = B_j^T B_j (symmetric
// tridiagonal, T[c][c] = alpha_{c+1}^2 + beta_{c+2}^2, T[c][c+1] =
// alpha_{c+2} beta_{c+2}):
//  * eigenvalues by multisection: each of the k largest is bracketed by
//    Sturm counts of the pivots d_c(x) of T - x I, many shifts per round in
//    parallel;
//  * the last component of each eigenvector from q[n-1]^2 = -1 / d'_{n-1}(lambda),
//    where d' follows by differentiating the pivot recurrence (det(T - x I) =
//    prod d_c(x), and the adjugate of T - lambda I at a simple eigenvalue);
//  * the residual bound alpha_{j+1} beta_{j+1} |q[n-1]| / omega (eq. lbdiagm2);
//  * final vectors by inverse iteration (one thread per vector) followed by
//    modified Gram-Schmidt across the k vectors.
#include <hip/hip_runtime.h>

#include "ssa_batch.h"

namespace ssa {
namespace batch {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

__device__ __forceinline__ float gaussian(unsigned long long seed, unsigned long long ctr, long long t) {
    uint32_t c[4] = {(uint32_t)t, (uint32_t)((unsigned long long)t >> 32), (uint32_t)ctr, (uint32_t)(ctr >> 32)};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967296.0);
    const double u2 = (double)c[1] * (1.0 / 4294967296.0);
    return (float)(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
}

// ---------------------------------------------------------------------------
// workgroup helpers

struct Ctx {
    Shared* sh;
    int tid;
    // series
    long long N, Li, Ki;  // internal window Li <= Ki
    int Mp, tw_shift;
    unsigned long long seed;
    // slot
    float* Ub;
    float* Vb;
    long long ld;
    float4* AB;
    double* scratch;  // inverse-iteration work, k * 6 * (kDmax + 2) doubles
    double* P;
    double* Q;
};

__device__ double block_sum(Ctx& c, double v) {
    v = wsum(v);
    const int lane = c.tid & 63, wave = c.tid >> 6;
    __syncthreads();
    if (lane == 0) c.sh->misc[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += c.sh->misc[w];
    __syncthreads();
    return s;
}

__device__ double block_max(Ctx& c, double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    const int lane = c.tid & 63, wave = c.tid >> 6;
    __syncthreads();
    if (lane == 0) c.sh->misc[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s = fmax(s, c.sh->misc[w]);
    __syncthreads();
    return s;
}

__device__ void fft(Ctx& c, int dir) {
    const TwoLevelTw tw{c.sh->tw_hi, c.sh->tw_lo, c.tw_shift};
    if (dir < 0)
        lds_fft_tw<-1, kEpt>(c.sh->buf, c.sh->st, 1, c.Mp, tw, c.tid, kThreads);
    else
        lds_fft_tw<1, kEpt>(c.sh->buf, c.sh->st, 1, c.Mp, tw, c.tid, kThreads);
}

// element m of the real sequence packed in buf (w[2n] + i w[2n+1] at buf[n])
__device__ __forceinline__ float getr(const float2* buf, long long m) {
    const float2 z = buf[m >> 1];
    return (m & 1) ? z.y : z.x;
}
__device__ __forceinline__ void setr(float2* buf, long long m, float v) {
    if (m & 1)
        buf[m >> 1].y = v;
    else
        buf[m >> 1].x = v;
}

// FFT length, radix plan and twiddle tables of one series
__device__ void setup_series_fft(Ctx& c) {
    long long mp = (c.N + 1) / 2;
    for (;; ++mp) {
        long long m = mp;
        for (int p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        if (m == 1) break;
    }
    c.Mp = (int)mp;
    if (c.tid == 0) {
        FftStages& st = c.sh->st;
        st.n = c.Mp;
        st.nstages = 0;
        int m = c.Mp;
        while (m % 8 == 0) { st.radix[st.nstages++] = 8; m /= 8; }
        while (m % 4 == 0) { st.radix[st.nstages++] = 4; m /= 4; }
        while (m % 2 == 0) { st.radix[st.nstages++] = 2; m /= 2; }
        for (int p : {3, 5, 7})
            while (m % p == 0) { st.radix[st.nstages++] = p; m /= p; }
    }
    int shift = 0;
    while ((1LL << (2 * shift)) < c.Mp) ++shift;
    c.tw_shift = shift;
    const int S = 1 << shift, nhi = (c.Mp + S - 1) / S;
    for (int t = c.tid; t < S || t < nhi; t += kThreads) {
        double sn, cs;
        if (t < S) {
            sincospi(-2.0 * (double)t / (double)c.Mp, &sn, &cs);
            c.sh->tw_lo[t] = make_float2((float)cs, (float)sn);
        }
        if (t < nhi) {
            sincospi(-2.0 * (double)((long long)t * S) / (double)c.Mp, &sn, &cs);
            c.sh->tw_hi[t] = make_float2((float)cs, (float)sn);
        }
    }
    __syncthreads();
}

// Spectral operator of the series: packed output Q(k) = A Z(k) + B conj Z(M'-k)
// for the circular convolution with the zero-padded series (natural order here).
__device__ void embed(Ctx& c, const double* f) {
    float2* buf = c.sh->buf;
    for (int n = c.tid; n < c.Mp; n += kThreads) {
        const long long m0 = 2LL * n, m1 = m0 + 1;
        buf[n] = make_float2(m0 < c.N ? (float)f[m0] : 0.0f, m1 < c.N ? (float)f[m1] : 0.0f);
    }
    __syncthreads();
    fft(c, -1);
    const double invMp = 1.0 / (double)c.Mp;
    const double M = 2.0 * c.Mp;
    for (int k = c.tid; k < c.Mp; k += kThreads) {
        const int kp = k == 0 ? 0 : c.Mp - k;
        const float2 z = buf[k], zp = buf[kp];
        const double er = 0.5 * ((double)z.x + (double)zp.x), ei = 0.5 * ((double)z.y - (double)zp.y);
        const double orr = 0.5 * ((double)z.y + (double)zp.y), oi = -0.5 * ((double)z.x - (double)zp.x);
        double sn, cs;
        sincospi(2.0 * (double)k / M, &sn, &cs);
        const double wor = cs * orr + sn * oi, woi = cs * oi - sn * orr;
        const double ar = (er - sn * wor) * invMp, ai = (ei - sn * woi) * invMp;
        const double br = -cs * woi * invMp, bi = cs * wor * invMp;
        c.AB[k] = make_float4((float)ar, (float)ai, (float)br, (float)bi);
    }
    __syncthreads();
}

// r = X x or X^T x as a convolution (x: n_in entries in global memory), minus
// coef * prev; r stays in buf, r[t] at real position n_in - 1 + t.
__device__ void convolve(Ctx& c, const float* x, long long n_in, long long n_out, const float* prev, double coef) {
    float2* buf = c.sh->buf;
    for (int n = c.tid; n < c.Mp; n += kThreads) {
        const long long m0 = 2LL * n, m1 = m0 + 1;
        buf[n] = make_float2(m0 < n_in ? x[n_in - 1 - m0] : 0.0f, m1 < n_in ? x[n_in - 1 - m1] : 0.0f);
    }
    __syncthreads();
    fft(c, -1);
    for (int k = c.tid; k <= c.Mp / 2; k += kThreads) {
        const int kp = k == 0 ? 0 : c.Mp - k;
        const float2 z0 = buf[k], z1 = buf[kp];
        const float4 o0 = c.AB[k], o1 = c.AB[kp];
        const float2 q0 = cadd(cmul(make_float2(o0.x, o0.y), z0), cmul(make_float2(o0.z, o0.w), cconj(z1)));
        const float2 q1 = cadd(cmul(make_float2(o1.x, o1.y), z1), cmul(make_float2(o1.z, o1.w), cconj(z0)));
        buf[k] = q0;
        if (kp != k) buf[kp] = q1;
    }
    __syncthreads();
    fft(c, 1);
    if (prev) {
        const float cf = (float)coef;
        for (long long t = c.tid; t < n_out; t += kThreads) {
            const long long m = n_in - 1 + t;
            setr(buf, m, getr(buf, m) - cf * prev[t]);
        }
    }
    __syncthreads();
}

// h[cc] = <basis_cc, r> for cc < ncols and h[ncols] = |r|^2, FP64 (exact
// FP32 x FP32 products), fixed reduction order.  r[t] = buf real position pos0 + t.
__device__ void project(Ctx& c, const float* basis, int ncols, long long n, long long pos0) {
    const float2* buf = c.sh->buf;
    const int lane = c.tid & 63, wave = c.tid >> 6;
    constexpr int G = 8;
    for (int c0 = 0; c0 <= ncols; c0 += G) {
        double acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.0;
        for (long long t = c.tid; t < n; t += kThreads) {
            const double r = (double)getr(buf, pos0 + t);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int cc = c0 + g;
                if (cc < ncols)
                    acc[g] += (double)basis[(long long)cc * c.ld + t] * r;
                else if (cc == ncols)
                    acc[g] += r * r;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double v = wsum(acc[g]);
            if (lane == 0 && c0 + g <= ncols) c.sh->red[wave][c0 + g] = v;
        }
    }
    __syncthreads();
    for (int cc = c.tid; cc <= ncols; cc += kThreads) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += c.sh->red[w][cc];
        c.sh->h[cc] = s;
    }
    __syncthreads();
}

// r -= basis h (in buf)
__device__ void subtract(Ctx& c, const float* basis, int ncols, long long n, long long pos0) {
    float2* buf = c.sh->buf;
    for (long long t = c.tid; t < n; t += kThreads) {
        double acc = (double)getr(buf, pos0 + t);
        for (int cc = 0; cc < ncols; ++cc) acc -= (double)basis[(long long)cc * c.ld + t] * c.sh->h[cc];
        setr(buf, pos0 + t, (float)acc);
    }
    __syncthreads();
}

// Coefficients and normalization of the new basis vector (r in buf); returns
// the B entry.  Same rules as the single-series path: one classical
// Gram-Schmidt pass with |r_new|^2 = |r|^2 - |h|^2, a second pass by the DGKS
// criterion, and a seeded random restart on breakdown.
__device__ double orthonormalize(Ctx& c, float* basis, int ncols, long long n, long long pos0,
                                 unsigned long long ctr, double* bnorm, int* restarts, int* dgks) {
    float2* buf = c.sh->buf;
    project(c, basis, ncols, n, pos0);
    double coef = 0.0, scale = 0.0;
    if (ncols >= n) {  // the basis already spans the space
        for (int cc = c.tid; cc < ncols; cc += kThreads) c.sh->h[cc] = 0.0;
        __syncthreads();
    } else {
        double hh = 0.0;
        for (int cc = c.tid; cc < ncols; cc += kThreads) hh += c.sh->h[cc] * c.sh->h[cc];
        hh = block_sum(c, hh);
        const double rr = c.sh->h[ncols];
        double a2 = rr - hh;
        const double thr = kBreakdownTol * *bnorm;
        if (a2 >= 0.5 * rr && sqrt(a2) > thr) {
            coef = sqrt(a2);
            scale = 1.0 / coef;
        } else {
            subtract(c, basis, ncols, n, pos0);
            project(c, basis, ncols, n, pos0);
            double hh2 = 0.0;
            for (int cc = c.tid; cc < ncols; cc += kThreads) hh2 += c.sh->h[cc] * c.sh->h[cc];
            hh2 = block_sum(c, hh2);
            a2 = c.sh->h[ncols] - hh2;
            if (a2 > 0.0 && sqrt(a2) > thr) {
                coef = sqrt(a2);
                scale = 1.0 / coef;
                ++*dgks;
            } else {
                for (long long t = c.tid; t < n; t += kThreads) setr(buf, pos0 + t, gaussian(c.seed, ctr, t));
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    project(c, basis, ncols, n, pos0);
                    subtract(c, basis, ncols, n, pos0);
                }
                project(c, basis, 0, n, pos0);
                const double r3 = c.sh->h[0];
                for (int cc = c.tid; cc < ncols; cc += kThreads) c.sh->h[cc] = 0.0;
                __syncthreads();
                scale = r3 > 0.0 ? 1.0 / sqrt(r3) : 0.0;
                ++*restarts;
            }
        }
    }
    // v = (r - basis h) * scale -> basis column ncols
    float* out = basis + (long long)ncols * c.ld;
    for (long long t = c.tid; t < n; t += kThreads) {
        double acc = (double)getr(buf, pos0 + t);
        for (int cc = 0; cc < ncols; ++cc) acc -= (double)basis[(long long)cc * c.ld + t] * c.sh->h[cc];
        out[t] = (float)(acc * scale);
    }
    if (coef > *bnorm) *bnorm = coef;
    __syncthreads();
    return coef;
}

// Sturm count of T - x I: number of eigenvalues < x
__device__ int sturm_count(const double* D, const double* E2, int n, double x, double pivmin) {
    double q = D[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        q = D[i] - x - E2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0 ? 1 : 0;
    }
    return cnt;
}

// The k largest eigenvalues of T_n (= omega^2) by multisection, and the squared
// last components of their eigenvectors; results in sh->lam[i], sh->qlast[i].
__device__ void tridiag_top(Ctx& c, int n, int k) {
    Shared* sh = c.sh;
    double* D = sh->tri;
    double* E2 = sh->tri + kDmax + 2;
    for (int i = c.tid; i < n; i += kThreads) {
        const double a = sh->alpha[i + 1], b = sh->beta[i + 2];
        D[i] = a * a + b * b;
        if (i + 1 < n) {
            const double e = sh->alpha[i + 2] * sh->beta[i + 2];
            E2[i] = e * e;
        }
    }
    __syncthreads();
    double g = 0.0, e2max = 0.0;
    for (int i = c.tid; i < n; i += kThreads) {
        const double el = i > 0 ? sqrt(E2[i - 1]) : 0.0, er = i + 1 < n ? sqrt(E2[i]) : 0.0;
        g = fmax(g, D[i] + el + er);
        if (i + 1 < n) e2max = fmax(e2max, E2[i]);
    }
    const double gmax = block_max(c, g);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, block_max(c, e2max));
    const int P = kThreads / k;  // shifts per eigenvalue per round
    for (int i = c.tid; i < k; i += kThreads) {
        sh->lo[i] = 0.0;
        sh->hi[i] = gmax * (1.0 + 1e-12) + 1e-300;
    }
    __syncthreads();
    const int ei = c.tid / P, p = c.tid % P;
    for (int round = 0; round < 14; ++round) {
        if (ei < k) {
            const double a = sh->lo[ei], b = sh->hi[ei];
            const double x = a + (b - a) * (double)(p + 1) / (double)(P + 1);
            sh->cnt[c.tid] = sturm_count(D, E2, n, x, pivmin);
            sh->xs[c.tid] = x;
        }
        __syncthreads();
        if (ei < k && p == 0) {
            const int m = n - 1 - ei;  // the eigenvalue is the m-th smallest
            double a = sh->lo[ei], b = sh->hi[ei];
            for (int q = 0; q < P; ++q) {
                const int idx = ei * P + q;
                if (sh->cnt[idx] <= m) {
                    a = sh->xs[idx];
                } else {
                    b = sh->xs[idx];
                    break;
                }
            }
            sh->lo[ei] = a;
            sh->hi[ei] = b;
        }
        __syncthreads();
    }
    for (int i = c.tid; i < k; i += kThreads) {
        const double lam = 0.5 * (sh->lo[i] + sh->hi[i]);
        sh->lam[i] = lam;
        // q[n-1]^2 = -1 / d'_{n-1}(lambda)
        double d = D[0] - lam, dp = -1.0;
        if (fabs(d) < pivmin) d = -pivmin;
        for (int j = 1; j < n; ++j) {
            const double t = E2[j - 1] / d;
            dp = -1.0 + t * dp / d;
            d = D[j] - lam - t;
            if (fabs(d) < pivmin) d = -pivmin;
        }
        sh->qlast[i] = dp < 0.0 ? fmin(1.0, -1.0 / dp) : 1.0;
    }
    __syncthreads();
}

// Stopping test on B_jj (alpha[1..jj+1], beta[2..jj+1] in LDS); thread 0 decides.
__device__ bool stopping_test(Ctx& c, int jj, int k, double tol, bool& have_prev, bool exhausted) {
    Shared* sh = c.sh;
    tridiag_top(c, jj, k);
    if (c.tid == 0) {
        const double w0 = sqrt(fmax(sh->lam[0], 0.0));
        bool ok = have_prev;
        for (int i = 0; i < k; ++i) {
            const double w = sqrt(fmax(sh->lam[i], 0.0));
            const double res = w > 0.0 ? sh->alpha[jj + 1] * sh->beta[jj + 1] * sqrt(sh->qlast[i]) / w : 0.0;
            const double sc = fmax(w, kResidFloor * w0);
            if (res > tol * sc) ok = false;
            if (fabs(w - sh->wprev[i]) > 10.0 * tol * sc) ok = false;
            sh->wprev[i] = w;
            sh->resid[i] = res;
        }
        if (exhausted) ok = true;
        sh->imisc[1] = ok ? 1 : 0;
    }
    __syncthreads();
    have_prev = true;
    const bool ok = sh->imisc[1] != 0;
    __syncthreads();
    return ok;
}

// Solve (T - lam I) x = x in place (partial pivoting; tiny pivots replaced).
__device__ void shifted_solve(const double* D, const double* E, int n, double lam, double tnorm, double* x,
                              double* a, double* b, double* cc, double* u2) {
    for (int i = 0; i < n; ++i) a[i] = D[i] - lam;
    for (int i = 0; i + 1 < n; ++i) {
        b[i] = E[i];
        cc[i] = E[i];
    }
    const double tiny = 2.220446049250313e-16 * (tnorm > 0.0 ? tnorm : 1.0);
    for (int i = 0; i + 1 < n; ++i) {
        u2[i] = 0.0;
        if (fabs(a[i]) >= fabs(cc[i])) {
            if (a[i] == 0.0) a[i] = tiny;
            const double f = cc[i] / a[i];
            a[i + 1] -= f * b[i];
            x[i + 1] -= f * x[i];
        } else {
            const double f = a[i] / cc[i];
            a[i] = cc[i];
            const double t = a[i + 1];
            a[i + 1] = b[i] - f * t;
            if (i + 2 < n) {
                u2[i] = b[i + 1];
                b[i + 1] = -f * b[i + 1];
            }
            b[i] = t;
            const double r0 = x[i];
            x[i] = x[i + 1];
            x[i + 1] = r0 - f * x[i + 1];
        }
    }
    if (a[n - 1] == 0.0) a[n - 1] = tiny;
    x[n - 1] /= a[n - 1];
    if (n >= 2) x[n - 2] = (x[n - 2] - b[n - 2] * x[n - 1]) / a[n - 2];
    for (int i = n - 3; i >= 0; --i) x[i] = (x[i] - b[i] * x[i + 1] - u2[i] * x[i + 2]) / a[i];
}

// Ritz coefficient matrices of B_d: Q (d x k) and P ((d+1) x k), row-major in
// global scratch, from the eigenvalues left in sh->lam by the last test.
__device__ void ritz_coefficients(Ctx& c, int d, int k) {
    Shared* sh = c.sh;
    double* D = sh->tri;
    double* E = sh->tri + kDmax + 2;  // off-diagonal (not squared) for the solves
    for (int i = c.tid; i < d; i += kThreads) {
        const double a = sh->alpha[i + 1], b = sh->beta[i + 2];
        D[i] = a * a + b * b;
        if (i + 1 < d) E[i] = sh->alpha[i + 2] * sh->beta[i + 2];
    }
    __syncthreads();
    double g = 0.0;
    for (int i = c.tid; i < d; i += kThreads) g = fmax(g, fabs(D[i]) + 2.0 * (i + 1 < d ? fabs(E[i]) : 0.0));
    const double tnorm = block_max(c, g);
    const long long stride = kDmax + 2;
    if (c.tid < k && c.tid < d) {
        const int i = c.tid;
        double* x = c.scratch + (long long)i * 6 * stride;
        double* a = x + stride;
        double* b = a + stride;
        double* cc = b + stride;
        double* u2 = cc + stride;
        for (int t = 0; t < d; ++t) x[t] = 1.0 + 0.5 * sin(0.7 * (t + 1) + 1.3 * (i + 1));
        for (int it = 0; it < 4; ++it) {
            shifted_solve(D, E, d, sh->lam[i], tnorm, x, a, b, cc, u2);
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
    __threadfence_block();
    __syncthreads();
    // modified Gram-Schmidt across the k vectors (handles equal eigenvalues)
    const int kk = k < d ? k : d;
    for (int i = 0; i < kk; ++i) {
        double* xi = c.scratch + (long long)i * 6 * stride;
        for (int p = 0; p < i; ++p) {
            const double* xp = c.scratch + (long long)p * 6 * stride;
            double dot = 0.0;
            for (int t = c.tid; t < d; t += kThreads) dot += xp[t] * xi[t];
            dot = block_sum(c, dot);
            for (int t = c.tid; t < d; t += kThreads) xi[t] -= dot * xp[t];
            __threadfence_block();
            __syncthreads();
        }
        double nrm = 0.0;
        for (int t = c.tid; t < d; t += kThreads) nrm += xi[t] * xi[t];
        nrm = sqrt(block_sum(c, nrm));
        for (int t = c.tid; t < d; t += kThreads) {
            xi[t] = nrm > 0.0 ? xi[t] / nrm : 0.0;
            c.Q[(long long)t * k + i] = xi[t];
        }
        __threadfence_block();
        __syncthreads();
        // p = B q / |B q|
        double pn = 0.0;
        for (int r = c.tid; r <= d; r += kThreads) {
            double v = 0.0;
            if (r < d) v += sh->alpha[r + 1] * xi[r];
            if (r >= 1) v += sh->beta[r + 1] * xi[r - 1];
            c.P[(long long)r * k + i] = v;
            pn += v * v;
        }
        pn = sqrt(block_sum(c, pn));
        for (int r = c.tid; r <= d; r += kThreads) c.P[(long long)r * k + i] = pn > 0.0 ? c.P[(long long)r * k + i] / pn : 0.0;
        __threadfence_block();
        __syncthreads();
    }
    for (int i = kk; i < k; ++i) {
        for (int t = c.tid; t < d; t += kThreads) c.Q[(long long)t * k + i] = 0.0;
        for (int r = c.tid; r <= d; r += kThreads) c.P[(long long)r * k + i] = 0.0;
    }
    __threadfence_block();
    __syncthreads();
}

// out[i*ldo + t] = sum_{cc < ncols} basis[cc][t] coef[cc*k + i], i < k
__device__ void ritz_vectors(Ctx& c, const float* basis, int ncols, const double* coef, int k, float* out,
                             long long ldo, long long n) {
    constexpr int T = 8;
    double* cs = &c.sh->red[0][0];  // ncols x T coefficients
    for (int i0 = 0; i0 < k; i0 += T) {
        for (int idx = c.tid; idx < ncols * T; idx += kThreads) {
            const int cc = idx / T, i = idx % T;
            cs[idx] = i0 + i < k ? coef[(long long)cc * k + i0 + i] : 0.0;
        }
        __syncthreads();
        for (long long t = c.tid; t < n; t += kThreads) {
            double acc[T];
#pragma unroll
            for (int i = 0; i < T; ++i) acc[i] = 0.0;
            for (int cc = 0; cc < ncols; ++cc) {
                const double x = basis[(long long)cc * c.ld + t];
#pragma unroll
                for (int i = 0; i < T; ++i) acc[i] += x * cs[cc * T + i];
            }
#pragma unroll
            for (int i = 0; i < T; ++i)
                if (i0 + i < k) out[(long long)(i0 + i) * ldo + t] = (float)acc[i];
        }
        __syncthreads();
    }
}

// Elementary series of one triple (Algorithm 4): g = sigma (u * v) / cnt.
// The packed spectrum of u waits in the slot's HBM scratch while v is
// transformed; each bin pair (k, M'-k) belongs to one thread, which reads both
// spectra there and writes the packed product back in place.
__device__ void hankelize(Ctx& c, double sigma, const float* u, long long lu, const float* v, long long lv,
                          float* out) {
    Shared* sh = c.sh;
    float2* buf = sh->buf;
    float2* zu = reinterpret_cast<float2*>(c.scratch);
    const long long N = c.N;
    const int Mp = c.Mp;
    const double M = 2.0 * Mp;
    for (int n = c.tid; n < Mp; n += kThreads) {
        const long long m0 = 2LL * n, m1 = m0 + 1;
        buf[n] = make_float2(m0 < lu ? u[m0] : 0.0f, m1 < lu ? u[m1] : 0.0f);
    }
    __syncthreads();
    fft(c, -1);
    for (int n = c.tid; n < Mp; n += kThreads) zu[n] = buf[n];
    __syncthreads();
    for (int n = c.tid; n < Mp; n += kThreads) {
        const long long m0 = 2LL * n, m1 = m0 + 1;
        buf[n] = make_float2(m0 < lv ? v[m0] : 0.0f, m1 < lv ? v[m1] : 0.0f);
    }
    __syncthreads();
    fft(c, -1);
    const double sc = sigma / (double)Mp;
    for (int k = c.tid; k <= Mp / 2; k += kThreads) {
        const int kp = k == 0 ? 0 : Mp - k;
        const float2 zu0 = zu[k], zu1 = zu[kp];
        const float2 zv0 = buf[k], zv1 = buf[kp];
        for (int side = 0; side < 2; ++side) {
            if (side == 1 && kp == k) break;
            const float2 a = side == 0 ? zu0 : zu1, ap = side == 0 ? zu1 : zu0;
            const float2 b = side == 0 ? zv0 : zv1, bp = side == 0 ? zv1 : zv0;
            const int kk = side == 0 ? k : kp;
            double sn, cs;
            sincospi(2.0 * (double)kk / M, &sn, &cs);
            const double wr = cs, wi = -sn;
            // E/O split, then the full spectra at kk and kk + M'
            const double uer = 0.5 * ((double)a.x + (double)ap.x), uei = 0.5 * ((double)a.y - (double)ap.y);
            const double uor = 0.5 * ((double)a.y + (double)ap.y), uoi = -0.5 * ((double)a.x - (double)ap.x);
            const double ver = 0.5 * ((double)b.x + (double)bp.x), vei = 0.5 * ((double)b.y - (double)bp.y);
            const double vor = 0.5 * ((double)b.y + (double)bp.y), voi = -0.5 * ((double)b.x - (double)bp.x);
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
    fft(c, 1);
    const long long L = lu, K = lv;
    for (long long m = c.tid; m < N; m += kThreads) {
        long long cnt = m + 1;
        if (L < cnt) cnt = L;
        if (K < cnt) cnt = K;
        if (N - m < cnt) cnt = N - m;
        if (cnt <= kEdge) {
            const long long a0 = m - K + 1 > 0 ? m - K + 1 : 0, a1 = m < L - 1 ? m : L - 1;
            double s = 0.0;
            for (long long aa = a0; aa <= a1; ++aa) s += (double)u[aa] * (double)v[m - aa];
            out[m] = (float)(sigma * s / (double)cnt);
        } else {
            out[m] = getr(buf, m) / (float)cnt;
        }
    }
    __syncthreads();
}

__device__ void solve_series(const BatchArgs& a, int s, Ctx& c) {
    Shared* sh = c.sh;
    const long long off = a.offs[s];
    const long long N = a.offs[s + 1] - off;
    const long long L = a.Ls[s], K = N - L + 1;
    const int k = a.ks[s];
    const bool transposed = L > K;
    c.N = N;
    c.Li = transposed ? K : L;
    c.Ki = transposed ? L : K;
    c.seed = a.seed ^ (0x9E3779B97F4A7C15ULL * (unsigned long long)(s + 1));
    setup_series_fft(c);
    embed(c, a.series + off);
    const long long Li = c.Li, Ki = c.Ki;
    for (int i = c.tid; i < kDmax + 3; i += kThreads) {
        sh->alpha[i] = 0.0;
        sh->beta[i] = 0.0;
    }
    for (int i = c.tid; i < kMaxK; i += kThreads) sh->wprev[i] = 0.0;
    double bnorm = 0.0;
    int restarts = 0, dgks = 0;
    // start vector (Algorithm 1, first line)
    for (long long t = c.tid; t < Li; t += kThreads) setr(sh->buf, t, gaussian(c.seed, 0, t));
    __syncthreads();
    {
        double dummy = 0.0;
        const double b1 = orthonormalize(c, c.Ub, 0, Li, 0, 1, &dummy, &restarts, &dgks);
        if (c.tid == 0) sh->beta[1] = b1;
    }
    const long long r_ = Li < Ki ? Li : Ki;
    const int d_cap = (int)(a.d_max < r_ ? a.d_max : r_);
    bool have_prev = false;
    int d = 0;
    bool conv = false;
    for (int j = 1;; ++j) {
        __syncthreads();
        convolve(c, c.Ub + (long long)(j - 1) * c.ld, Li, Ki, j >= 2 ? c.Vb + (long long)(j - 2) * c.ld : nullptr,
                 sh->beta[j]);
        const double aj = orthonormalize(c, c.Vb, j - 1, Ki, Li - 1, 2ULL * j, &bnorm, &restarts, &dgks);
        if (c.tid == 0) sh->alpha[j] = aj;
        __syncthreads();
        const int jj = j - 1;
        if (jj >= k && (jj % a.check_every == 0 || jj >= d_cap)) {
            const bool exhausted = jj >= r_;
            const bool ok = stopping_test(c, jj, k, a.tol, have_prev, exhausted);
            if (ok || jj >= d_cap) {
                d = jj;
                conv = ok;
                break;
            }
        }
        convolve(c, c.Vb + (long long)(j - 1) * c.ld, Ki, Li, c.Ub + (long long)(j - 1) * c.ld, sh->alpha[j]);
        const double bj = orthonormalize(c, c.Ub, j, Li, Ki - 1, 2ULL * j + 1, &bnorm, &restarts, &dgks);
        if (c.tid == 0) sh->beta[j + 1] = bj;
        __syncthreads();
    }
    // Ritz triples
    ritz_coefficients(c, d, k);
    float* Uo = a.U + a.uoff[s];
    float* Vo = a.V + a.voff[s];
    float* Ui = transposed ? Vo : Uo;  // internal U has Li entries
    float* Vi = transposed ? Uo : Vo;
    ritz_vectors(c, c.Ub, d + 1, c.P, k, Ui, Li, Li);
    ritz_vectors(c, c.Vb, d, c.Q, k, Vi, Ki, Ki);
    for (int i = c.tid; i < k; i += kThreads) a.sigma[a.soff[s] + i] = sqrt(fmax(sh->lam[i], 0.0));
    if (c.tid == 0 && a.info) {
        int* inf = a.info + 4LL * s;
        inf[0] = d;
        inf[1] = conv ? 1 : 0;
        inf[2] = restarts;
        inf[3] = dgks;
    }
    __threadfence_block();
    __syncthreads();
    if (a.recon) {
        for (int i = 0; i < k; ++i) {
            const double sg = sqrt(fmax(sh->lam[i], 0.0));
            hankelize(c, sg, Uo + (long long)i * L, L, Vo + (long long)i * K, K, a.recon + a.roff[s] + (long long)i * N);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs a) {
    extern __shared__ char lds[];
    Ctx c;
    c.sh = reinterpret_cast<Shared*>(lds);
    c.tid = threadIdx.x;
    char* slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
    c.ld = a.ld;
    c.AB = reinterpret_cast<float4*>(slot + a.o_ab);
    c.Ub = reinterpret_cast<float*>(slot + a.o_u);
    c.Vb = reinterpret_cast<float*>(slot + a.o_v);
    c.scratch = reinterpret_cast<double*>(slot + a.o_scratch);
    c.P = reinterpret_cast<double*>(slot + a.o_p);
    c.Q = reinterpret_cast<double*>(slot + a.o_q);
    for (;;) {
        if (c.tid == 0) c.sh->imisc[0] = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int s = c.sh->imisc[0];
        __syncthreads();
        if (s >= a.nseries) break;
        solve_series(a, s, c);
    }
}

}  // namespace batch

hipError_t launch_batch(const BatchArgs& a, int nslots, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch::k_batch),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)sizeof(batch::Shared));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(batch::k_batch, dim3(nslots), dim3(batch::kThreads), sizeof(batch::Shared), s, a);
    return hipGetLastError();
}

size_t batch_lds_bytes() { return sizeof(batch::Shared); }

}  // namespace ssa
