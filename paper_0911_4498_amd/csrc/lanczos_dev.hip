// lanczos_dev.hip -- the stopping test and the Ritz coefficients of the
// single-series solver, on the device (Sec. 3.1, eqs. lbdiagm1/lbdiagm2).
//
// B_j is (j+1) x j lower bidiagonal (alpha on the diagonal, beta below it).  Its
// right singular vectors are the eigenvectors of T = B_j^T B_j, a symmetric
// tridiagonal (the cross-product form of Theorem 1), and the residual of Ritz
// triple i is alpha_{j+1} beta_{j+1} |q_i[j-1]| / omega_i.
//  * k_lz_eig (one workgroup per triple) finds eigenvalue i of T by multisection
//    on Sturm counts, 512 shifts per round, and the last component of its
//    eigenvector by a twisted factorization;
//  * k_lz_decide applies the stopping rule and writes a small record, the only
//    data the host reads back;
//  * k_lz_invit (one workgroup per triple) turns the final eigenvalues into
//    eigenvectors q_i by inverse iteration, and k_lz_orth makes them orthonormal
//    and forms P = B Q Omega^-1, completed to an orthonormal set where omega = 0
//    (the _lds versions hold every work array in LDS; the plain ones, for bases too
//    long for that, work in global memory).
// The Lanczos scalars never leave the device.
#include <hip/hip_runtime.h>

#include "ssa_internal.h"
#include "tridiag_dev.h"

namespace ssa {

// Sturm counts at two shifts at once (two independent pivot chains interleaved).
__device__ __forceinline__ void sturm_count2(const double* D, const double* E2, int n, double x0, double x1,
                                             double pivmin, int& c0, int& c1) {
    double q0 = D[0] - x0, q1 = D[0] - x1;
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    c0 = q0 < 0.0 ? 1 : 0;
    c1 = q1 < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        const double d = D[i], e = E2[i - 1];
        q0 = (d - x0) - e * fast_rcp(q0);
        q1 = (d - x1) - e * fast_rcp(q1);
        if (fabs(q0) < pivmin) q0 = -pivmin;
        if (fabs(q1) < pivmin) q1 = -pivmin;
        c0 += q0 < 0.0 ? 1 : 0;
        c1 += q1 < 0.0 ? 1 : 0;
    }
}

constexpr int kEigThreads = 256;          // 2 shifts per thread: 512 per round
constexpr int kEigShifts = 2 * kEigThreads;
constexpr int kEigRounds = 6;             // 513^6 > 2^54: a bracket of width gmax shrinks below 2^-54 gmax

// Eigenvalue i = blockIdx.x (the i-th largest) of T = B_jj^T B_jj and the squared last
// component of its eigenvector: multisection with 512 shifts per round from [0, gmax],
// then the twisted factorization (Dhillon and Parlett) at the midpoint.  Results go to
// scr[i] (eigenvalue) and scr[kstride + i] (squared last component).
__global__ __launch_bounds__(kEigThreads) void k_lz_eig(LzCheck a) {
    extern __shared__ double sm[];
    if (a.rec[kChkDone] != 0.0) return;
    const int tid = threadIdx.x, n = a.jj, i = blockIdx.x;
    double* D = sm;                   // n
    double* E2 = D + n;               // n
    double* xs = E2 + n;              // kEigShifts
    double* misc = xs + kEigShifts;   // 8
    int* cnt = reinterpret_cast<int*>(misc + 8);  // kEigShifts
    for (int t = tid; t < n; t += kEigThreads) {
        const double x = a.alpha[t + 1], y = a.beta[t + 2];
        D[t] = x * x + y * y;
        const double e = t + 1 < n ? a.alpha[t + 2] * a.beta[t + 2] : 0.0;
        E2[t] = e * e;
    }
    __syncthreads();
    double g = 0.0, e2max = 0.0;
    for (int t = tid; t < n; t += kEigThreads) {
        const double el = t > 0 ? sqrt(E2[t - 1]) : 0.0, er = t + 1 < n ? sqrt(E2[t]) : 0.0;
        g = fmax(g, D[t] + el + er);
        if (t + 1 < n) e2max = fmax(e2max, E2[t]);
    }
    // workgroup maxima (4 waves)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        g = fmax(g, __shfl_down(g, off, 64));
        e2max = fmax(e2max, __shfl_down(e2max, off, 64));
    }
    if ((tid & 63) == 0) {
        misc[tid >> 6] = g;
        misc[4 + (tid >> 6)] = e2max;
    }
    __syncthreads();
    const double gmax = fmax(fmax(misc[0], misc[1]), fmax(misc[2], misc[3]));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, fmax(fmax(misc[4], misc[5]), fmax(misc[6], misc[7])));
    __syncthreads();
    const int m = n - 1 - i;  // the eigenvalue is the m-th smallest
    double lo = 0.0, hi = gmax * (1.0 + 1e-12) + 1e-300;
    for (int round = 0; round < kEigRounds; ++round) {
        const double w = (hi - lo) / (double)(kEigShifts + 1);
        const double x0 = lo + w * (double)(2 * tid + 1), x1 = lo + w * (double)(2 * tid + 2);
        int c0, c1;
        sturm_count2(D, E2, n, x0, x1, pivmin, c0, c1);
        xs[2 * tid] = x0;
        xs[2 * tid + 1] = x1;
        cnt[2 * tid] = c0;
        cnt[2 * tid + 1] = c1;
        __syncthreads();
        // the first shift with more than m eigenvalues below it bounds lambda from above
        int first = kEigShifts;
        for (int t = tid; t < kEigShifts; t += kEigThreads)
            if (cnt[t] > m) first = min(first, t);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) first = min(first, __shfl_down(first, off, 64));
        if ((tid & 63) == 0) cnt[kEigShifts + (tid >> 6)] = first;
        __syncthreads();
        first = min(min(cnt[kEigShifts], cnt[kEigShifts + 1]), min(cnt[kEigShifts + 2], cnt[kEigShifts + 3]));
        const double nlo = first > 0 ? xs[first - 1] : lo;
        const double nhi = first < kEigShifts ? xs[first] : hi;
        lo = nlo;
        hi = nhi;
        __syncthreads();
    }
    if (tid == 0) {
        const double lam = 0.5 * (lo + hi);
        double* dm = a.scr + 2 * a.kstride + (long long)i * 2 * a.dstride;
        a.scr[i] = lam;
        a.scr[a.kstride + i] = twisted_qlast<true>(D, E2, n, lam, pivmin, dm, dm + a.dstride);
    }
}

// The stopping rule on the k eigenvalues and last components left by k_lz_eig: every
// residual bound <= tol * max(omega_i, 1e-5 omega_1) and the k Ritz values within
// 10 tol (relative) of the previous test's; or the Krylov space exhausted (B exact); or
// the step cap.  Once the record says done, later tests (steps enqueued ahead of the
// host's decision) return at once.
__global__ void k_lz_decide(LzCheck a) {
    double* rec = a.rec;
    if (threadIdx.x != 0 || rec[kChkDone] != 0.0) return;
    const int n = a.jj, k = a.k;
    double* lam = rec + kChkHdr;
    double* wprev = lam + a.kstride;
    double* resid = wprev + a.kstride;
    const double* el = a.scr;
    const double* ql = a.scr + a.kstride;
    const double w0 = sqrt(fmax(el[0], 0.0));
    bool ok = rec[kChkHavePrev] != 0.0;
    const double ab = a.alpha[n + 1] * a.beta[n + 1];
    for (int i = 0; i < k; ++i) {
        const double w = sqrt(fmax(el[i], 0.0));
        const double res = w > 0.0 ? ab * sqrt(ql[i]) / w : 0.0;
        const double sc = fmax(w, kResidFloorDev * w0);
        if (!(res <= a.tol * sc)) ok = false;
        if (!(fabs(w - wprev[i]) <= 10.0 * a.tol * sc)) ok = false;
        wprev[i] = w;
        resid[i] = res;
        lam[i] = el[i];
    }
    rec[kChkHavePrev] = 1.0;
    rec[kChkJJ] = (double)n;
    rec[kChkRestarts] = a.snap[0];
    rec[kChkDgks] = a.snap[1];
    const bool bad = a.nonfinite && *a.nonfinite != 0.0;
    if (bad) rec[kChkNonfinite] = 1.0;
    const bool exhausted = n >= a.rmin;
    if (ok || exhausted || n >= a.dcap || bad) {
        rec[kChkDone] = 1.0;
        rec[kChkD] = (double)n;
        rec[kChkConv] = (ok || exhausted) ? 1.0 : 0.0;
    }
}

// Inverse iteration for Ritz triple i = blockIdx.x: 4 solves of (T - lambda_i I) x = x
// from a fixed start (thread 0; tridiagonal LU with partial pivoting), normalized, into
// scr + i * 5 * dstride.
__global__ __launch_bounds__(64) void k_lz_invit(LzRitz a) {
    const int d = (int)a.rec[kChkD], i = blockIdx.x;
    if (threadIdx.x != 0 || i >= d) return;
    const double lam = a.rec[kChkHdr + i];
    const long long st = a.dstride;
    double* x = a.scr + (long long)i * 5 * st;
    double* D = x + st;      // diagonal and off-diagonal of T, then the solver's work arrays
    double* E = D + st;
    double* wa = E + st;
    double* wb = wa + st;
    // the solver overwrites its work arrays only: (a, b, cc, u2) = (wa, wb, E-copy, D-copy)
    double tnorm = 0.0;
    for (int t = 0; t < d; ++t) {
        const double al = a.alpha[t + 1], be = a.beta[t + 2];
        D[t] = al * al + be * be;
        E[t] = t + 1 < d ? a.alpha[t + 2] * a.beta[t + 2] : 0.0;
        tnorm = fmax(tnorm, fabs(D[t]) + 2.0 * fabs(E[t]));
        x[t] = 1.0 + 0.5 * sin(0.7 * (t + 1) + 1.3 * (i + 1));
    }
    double* cc = a.scr + (long long)a.k * 5 * st + (long long)i * 2 * st;  // two more work arrays
    double* u2 = cc + st;
    for (int it = 0; it < 4; ++it) {
        shifted_solve<true>(D, E, d, lam, tnorm, x, wa, wb, cc, u2);
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

__device__ __forceinline__ double wave_dot(const double* x, const double* y, int n, int lane) {
    double s = 0.0;
    for (int t = lane; t < n; t += 64) s += x[t] * y[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// The Ritz coefficient matrices from the inverse-iteration vectors, one wave: Q by
// modified Gram-Schmidt across the k vectors (two passes); P[:, i] = B Q[:, i], kept
// orthogonal to the earlier columns (two passes) and normalized, or a unit vector
// orthogonal to them where B Q[:, i] vanishes (omega_i = 0).  P ((d+1) x k) and Q
// (d x k) are row-major with row stride kstride; sigma_i = sqrt(lambda_i).
__global__ __launch_bounds__(64) void k_lz_orth(LzRitz a) {
    const int lane = threadIdx.x, k = a.k;
    const int d = (int)a.rec[kChkD];
    const double* lam = a.rec + kChkHdr;
    const long long st = a.dstride;
    const int kk = k < d ? k : d;
    double bmax = 0.0;
    for (int t = lane; t < d; t += 64) bmax = fmax(bmax, fmax(fabs(a.alpha[t + 1]), fabs(a.beta[t + 2])));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, off, 64));
    // left vectors are built in a scratch column block: p_i at pl + i * (d + 1)
    double* pl = a.scr + (long long)a.k * 7 * st;
    for (int i = 0; i < kk; ++i) {
        double* xi = a.scr + (long long)i * 5 * st;
        for (int pass = 0; pass < 2; ++pass)
            for (int p = 0; p < i; ++p) {
                const double* xp = a.scr + (long long)p * 5 * st;
                const double h = wave_dot(xp, xi, d, lane);
                for (int t = lane; t < d; t += 64) xi[t] -= h * xp[t];
            }
        const double nrm = sqrt(wave_dot(xi, xi, d, lane));
        for (int t = lane; t < d; t += 64) {
            xi[t] = nrm > 0.0 ? xi[t] / nrm : 0.0;
            a.Q[(long long)t * a.kstride + i] = xi[t];
        }
        double* pi = pl + (long long)i * (d + 1);
        for (int r = lane; r <= d; r += 64) {
            double v = 0.0;
            if (r < d) v += a.alpha[r + 1] * xi[r];
            if (r >= 1) v += a.beta[r + 1] * xi[r - 1];
            pi[r] = v;
        }
        double pn = 0.0;
        for (int c = d + 1;; --c) {  // c = d + 1: B q itself; then the unit vectors e_d, e_{d-1}, ...
            if (c <= d)
                for (int r = lane; r <= d; r += 64) pi[r] = r == c ? 1.0 : 0.0;
            for (int pass = 0; pass < 2; ++pass)
                for (int p = 0; p < i; ++p) {
                    const double* pp = pl + (long long)p * (d + 1);
                    const double h = wave_dot(pp, pi, d + 1, lane);
                    for (int r = lane; r <= d; r += 64) pi[r] -= h * pp[r];
                }
            pn = sqrt(wave_dot(pi, pi, d + 1, lane));
            if (c == d + 1 ? pn > 1e-12 * bmax : pn >= 0.5) break;
            if (c == 0) {
                pn = 0.0;
                break;
            }
        }
        for (int r = lane; r <= d; r += 64) {
            pi[r] = pn > 0.0 ? pi[r] / pn : 0.0;
            a.P[(long long)r * a.kstride + i] = pi[r];
        }
    }
    for (int i = lane; i < k; i += 64) a.sigma[i] = i < kk ? sqrt(fmax(lam[i], 0.0)) : 0.0;
}

// ---- the same Ritz coefficients with every work array in LDS ----------------------
// One eigenvector solve is a chain of dependent divisions; with its arrays in global
// memory each step also waits for a memory round trip.  These versions keep D, E, the
// iterate and the factors in LDS and carry the running row in registers.

constexpr int kInvitArrays = 8;           // D, E, x and the factor rows A, 1/A, Bv, U2, F
constexpr size_t kRitzLdsMax = 64 * 1024; // larger bases take the global-memory kernels
constexpr int kOrthThreads = 256;  // few waves: the orthonormalization is a chain of short phases
constexpr int kOrthWaves = kOrthThreads / 64;

size_t invit_lds_bytes(int d) { return (sizeof(double) * kInvitArrays + 1) * (size_t)d; }
size_t orth_lds_bytes(int d, int k) {
    const size_t kk = (size_t)(k < d ? k : d);
    return sizeof(double) * (kk * (size_t)d + kk * (size_t)(d + 1) + (size_t)k + kOrthWaves + 2 * (size_t)(d + 2));
}

// LU factorization of T - lam I (T = diagonal D, off-diagonal E) with partial pivoting,
// a zero pivot replaced by eps |T|: the elimination of shifted_solve with the row being
// eliminated carried in registers.  Row i of U goes to A (pivot; RA = its reciprocal),
// Bv and U2 (the fill-in of a row swap); F[i] is the multiplier and Sw[i] marks a swap.
// The factors do not depend on the right-hand side, so every inverse-iteration step
// reuses them (the same arithmetic as refactoring each time).
__device__ __forceinline__ void tri_factor(const double* __restrict__ D, const double* __restrict__ E, int n,
                                           double lam, double tnorm, double* __restrict__ A,
                                           double* __restrict__ RA, double* __restrict__ Bv,
                                           double* __restrict__ U2, double* __restrict__ F,
                                           unsigned char* __restrict__ Sw) {
    const double tiny = 2.220446049250313e-16 * (tnorm > 0.0 ? tnorm : 1.0);
    double ai = D[0] - lam, bi = n > 1 ? E[0] : 0.0;
#pragma unroll 4
    for (int i = 0; i + 1 < n; ++i) {
        const double ci = E[i];
        const double an = D[i + 1] - lam;  // next row, not yet touched
        const double bn = i + 2 < n ? E[i + 1] : 0.0;
        if (fabs(ai) >= fabs(ci)) {
            if (ai == 0.0) ai = tiny;
            const double r = fast_rcp(ai);
            const double f = ci * r;
            A[i] = ai;
            RA[i] = r;
            Bv[i] = bi;
            U2[i] = 0.0;
            F[i] = f;
            Sw[i] = 0;
            ai = an - f * bi;
            bi = bn;
        } else {  // rows i and i + 1 swap
            const double r = fast_rcp(ci);
            const double f = ai * r;
            A[i] = ci;
            RA[i] = r;
            Bv[i] = an;
            U2[i] = bn;
            F[i] = f;
            Sw[i] = 1;
            ai = bi - f * an;
            bi = -f * bn;
        }
    }
    if (ai == 0.0) ai = tiny;
    A[n - 1] = ai;
    RA[n - 1] = fast_rcp(ai);
}

// x <- (T - lam I)^{-1} x with the factors of tri_factor.
__device__ __forceinline__ void tri_apply(int n, const double* __restrict__ RA, const double* __restrict__ Bv,
                                          const double* __restrict__ U2, const double* __restrict__ F,
                                          const unsigned char* __restrict__ Sw, double* __restrict__ x) {
    double xi = x[0];
#pragma unroll 4
    for (int i = 0; i + 1 < n; ++i) {
        const double xn = x[i + 1];
        if (Sw[i]) {
            x[i] = xn;
            xi = xi - F[i] * xn;
        } else {
            x[i] = xi;
            xi = xn - F[i] * xi;
        }
    }
    double x1 = xi * RA[n - 1];  // x[i + 1] and x[i + 2] of the back substitution
    x[n - 1] = x1;
    if (n < 2) return;
    double x2 = x1;
    x1 = (x[n - 2] - Bv[n - 2] * x1) * RA[n - 2];
    x[n - 2] = x1;
#pragma unroll 4
    for (int i = n - 3; i >= 0; --i) {
        const double v = (x[i] - Bv[i] * x1 - U2[i] * x2) * RA[i];
        x[i] = v;
        x2 = x1;
        x1 = v;
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Inverse iteration for Ritz triple i = blockIdx.x (one wave): 4 solves from the fixed
// start of k_lz_invit, each normalized; the vector goes to scr + i * 5 * dstride.
__global__ __launch_bounds__(64) void k_lz_invit_lds(LzRitz a) {
    extern __shared__ double sm[];
    const int d = (int)a.rec[kChkD], i = blockIdx.x, lane = threadIdx.x;
    if (i >= d) return;
    const double lam = a.rec[kChkHdr + i];
    double* D = sm;
    double* E = D + d;
    double* x = E + d;
    double* A = x + d;
    double* RA = A + d;
    double* Bv = RA + d;
    double* U2 = Bv + d;
    double* F = U2 + d;
    unsigned char* Sw = reinterpret_cast<unsigned char*>(F + d);
    double tn = 0.0;
    for (int t = lane; t < d; t += 64) {
        const double al = a.alpha[t + 1], be = a.beta[t + 2];
        D[t] = al * al + be * be;
        E[t] = t + 1 < d ? a.alpha[t + 2] * a.beta[t + 2] : 0.0;
        tn = fmax(tn, fabs(D[t]) + 2.0 * fabs(E[t]));
        x[t] = 1.0 + 0.5 * sin(0.7 * (t + 1) + 1.3 * (i + 1));
    }
    tn = wave_max(tn);
    __syncthreads();
    if (lane == 0) tri_factor(D, E, d, lam, tn, A, RA, Bv, U2, F, Sw);
    __syncthreads();
    for (int it = 0; it < 4; ++it) {
        if (lane == 0) tri_apply(d, RA, Bv, U2, F, Sw, x);
        __syncthreads();
        double nrm = sqrt(wave_dot(x, x, d, lane));
        const bool bad = !(nrm > 0.0) || !isfinite(nrm);
        for (int t = lane; t < d; t += 64) x[t] = bad ? (t == i ? 1.0 : 0.0) : x[t] / nrm;
        __syncthreads();
    }
    double* out = a.scr + (long long)i * 5 * a.dstride;
    for (int t = lane; t < d; t += 64) out[t] = x[t];
}

// Sum over the workgroup in a fixed order (wave sums, then the kOrthWaves partials).
__device__ __forceinline__ double orth_block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    lds_barrier();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kOrthWaves; ++w) s += red[w];
    lds_barrier();
    return s;
}

// y -= sum_{p < m} <v_p, y> v_p, twice (classical Gram-Schmidt with one
// reorthogonalization), for the m vectors v_p = V + p * len in LDS.
__device__ __forceinline__ void orth_against(double* y, const double* V, int m, int len, double* hv) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int pass = 0; pass < 2; ++pass) {
        for (int q = wave; q < m; q += kOrthWaves) {
            const double h = wave_dot(V + (long long)q * len, y, len, lane);
            if (lane == 0) hv[q] = h;
        }
        lds_barrier();
        for (int t = tid; t < len; t += kOrthThreads) {
            double v = y[t];
            int q = 0;
            // four terms' loads ahead of their (in-order) subtractions
            for (; q + 4 <= m; q += 4) {
                const double h0 = hv[q], h1 = hv[q + 1], h2 = hv[q + 2], h3 = hv[q + 3];
                const double w0 = V[(long long)q * len + t], w1 = V[(long long)(q + 1) * len + t];
                const double w2 = V[(long long)(q + 2) * len + t], w3 = V[(long long)(q + 3) * len + t];
                v -= h0 * w0;
                v -= h1 * w1;
                v -= h2 * w2;
                v -= h3 * w3;
            }
            for (; q < m; ++q) v -= hv[q] * V[(long long)q * len + t];
            y[t] = v;
        }
        lds_barrier();
    }
}

// k_lz_orth with the vectors in LDS and the projections of one step in parallel.
__global__ __launch_bounds__(kOrthThreads) void k_lz_orth_lds(LzRitz a) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x, k = a.k;
    const int d = (int)a.rec[kChkD];
    const double* lam = a.rec + kChkHdr;
    const int kk = k < d ? k : d;
    double* Xq = sm;                        // kk vectors of length d
    double* Pl = Xq + (long long)kk * d;    // kk vectors of length d + 1
    double* hv = Pl + (long long)kk * (d + 1);
    double* red = hv + k;
    double* al = red + kOrthWaves;  // alpha[0 .. d+1], beta[0 .. d+1]
    double* be = al + d + 2;
    for (int t = tid; t < d + 2; t += kOrthThreads) {
        al[t] = a.alpha[t];
        be[t] = a.beta[t];
    }
    for (int i = 0; i < kk; ++i)
        for (int t = tid; t < d; t += kOrthThreads) Xq[(long long)i * d + t] = a.scr[(long long)i * 5 * a.dstride + t];
    lds_barrier();
    double bm = 0.0;
    for (int t = tid; t < d; t += kOrthThreads) bm = fmax(bm, fmax(fabs(al[t + 1]), fabs(be[t + 2])));
    bm = wave_max(bm);
    if ((tid & 63) == 0) red[tid >> 6] = bm;
    lds_barrier();
    double bmax = 0.0;
    for (int w = 0; w < kOrthWaves; ++w) bmax = fmax(bmax, red[w]);
    lds_barrier();
    for (int i = 0; i < kk; ++i) {
        double* xi = Xq + (long long)i * d;
        orth_against(xi, Xq, i, d, hv);
        double ss = 0.0;
        for (int t = tid; t < d; t += kOrthThreads) ss += xi[t] * xi[t];
        const double nrm = sqrt(orth_block_sum(ss, red));
        for (int t = tid; t < d; t += kOrthThreads) {
            const double v = nrm > 0.0 ? xi[t] / nrm : 0.0;
            xi[t] = v;
            a.Q[(long long)t * a.kstride + i] = v;
        }
        lds_barrier();
        double* pi = Pl + (long long)i * (d + 1);
        double pn = 0.0;
        for (int c = d + 1;; --c) {  // c = d + 1: B q itself; then the unit vectors e_d, e_{d-1}, ...
            for (int r = tid; r <= d; r += kOrthThreads) {
                double v = 0.0;
                if (c == d + 1) {
                    if (r < d) v += al[r + 1] * xi[r];
                    if (r >= 1) v += be[r + 1] * xi[r - 1];
                } else {
                    v = r == c ? 1.0 : 0.0;
                }
                pi[r] = v;
            }
            lds_barrier();
            orth_against(pi, Pl, i, d + 1, hv);
            double sp = 0.0;
            for (int r = tid; r <= d; r += kOrthThreads) sp += pi[r] * pi[r];
            pn = sqrt(orth_block_sum(sp, red));
            if (c == d + 1 ? pn > 1e-12 * bmax : pn >= 0.5) break;
            if (c == 0) {
                pn = 0.0;
                break;
            }
        }
        for (int r = tid; r <= d; r += kOrthThreads) {
            const double v = pn > 0.0 ? pi[r] / pn : 0.0;
            pi[r] = v;
            a.P[(long long)r * a.kstride + i] = v;
        }
        lds_barrier();
    }
    for (int i = tid; i < k; i += kOrthThreads) a.sigma[i] = i < kk ? sqrt(fmax(lam[i], 0.0)) : 0.0;
}

hipError_t launch_lz_check(const LzCheck& a, hipStream_t s) {
    const size_t lds = sizeof(double) * (2 * (size_t)a.jj + kEigShifts + 8) + sizeof(int) * (kEigShifts + 4);
    hipLaunchKernelGGL(k_lz_eig, dim3((unsigned)a.k), dim3(kEigThreads), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_decide, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

// d: the dimension the deciding test recorded (the host read it from the record).
hipError_t launch_lz_ritz(const LzRitz& a, int d, hipStream_t s) {
    const size_t li = invit_lds_bytes(d), lo = orth_lds_bytes(d, a.k);
    if (li <= kRitzLdsMax && lo <= kRitzLdsMax) {
        hipLaunchKernelGGL(k_lz_invit_lds, dim3((unsigned)a.k), dim3(64), li, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lz_orth_lds, dim3(1), dim3(kOrthThreads), lo, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_lz_invit, dim3((unsigned)a.k), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_orth, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t set_lz_attributes() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_lz_invit_lds),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRitzLdsMax);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_lz_orth_lds),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRitzLdsMax);
}

}  // namespace ssa
