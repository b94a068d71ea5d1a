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
//    eigenvectors q_i by inverse iteration, and k_lz_orth (one wave) makes them
//    orthonormal and forms P = B Q Omega^-1, completed to an orthonormal set where
//    omega = 0.
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
    rec[kChkRestarts] = a.state[1];
    rec[kChkDgks] = a.state[2];
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

hipError_t launch_lz_check(const LzCheck& a, hipStream_t s) {
    const size_t lds = sizeof(double) * (2 * (size_t)a.jj + kEigShifts + 8) + sizeof(int) * (kEigShifts + 4);
    hipLaunchKernelGGL(k_lz_eig, dim3((unsigned)a.k), dim3(kEigThreads), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_decide, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lz_ritz(const LzRitz& a, int d, hipStream_t s) {
    (void)d;
    hipLaunchKernelGGL(k_lz_invit, dim3((unsigned)a.k), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_orth, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ssa
