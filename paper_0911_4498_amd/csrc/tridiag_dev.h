// tridiag_dev.h -- device routines on the symmetric tridiagonal T = B^T B of a
// Lanczos bidiagonal B (Sec. 3.1; T[c][c] = alpha_{c+1}^2 + beta_{c+2}^2,
// T[c][c+1] = alpha_{c+2} beta_{c+2}): Sturm counts, the k largest eigenvalues by
// multisection, the last eigenvector components by twisted factorizations
// (the residual bounds of eqs. lbdiagm1/lbdiagm2), and shifted solves for inverse
// iteration.  Shared by the many-series engine and the single-series stopping test.
#pragma once
#include <hip/hip_runtime.h>

namespace ssa {

#ifndef SSA_TRI_INLINE
#define SSA_TRI_INLINE __device__ __attribute__((always_inline)) inline
#endif

// 1/q from the hardware reciprocal and one Newton step (relative error ~ 2^-52): the
// pivot recurrences below are chains of divisions, and this halves their latency.
SSA_TRI_INLINE double fast_rcp(double q) {
    double r = __builtin_amdgcn_rcp(q);
    const double e = fma(-q, r, 1.0);
    return fma(r, e, r);
}

// x / y, or x * fast_rcp(y) in the FAST instantiations
template <bool FAST>
SSA_TRI_INLINE double tri_div(double x, double y) {
    if constexpr (FAST)
        return x * fast_rcp(y);
    else
        return x / y;
}

// Number of eigenvalues below x of the tridiagonal with diagonal D and squared
// off-diagonal E2 (pivots of T - x I, tiny pivots replaced by -pivmin).
SSA_TRI_INLINE int sturm_count(const double* D, const double* E2, int n, double x, double pivmin) {
    double d = D[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    int cnt = d < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        d = D[i] - x - E2[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        cnt += d < 0.0 ? 1 : 0;
    }
    return cnt;
}

// The k largest eigenvalues of the n x n tridiagonal (D, E2), k <= NT: each round
// evaluates NT / k shifts per eigenvalue inside its bracket [lo[i], hi[i]] (set
// by the caller) and keeps the sub-interval holding it.  xs and cnt hold NT
// entries each (workgroup-shared memory); every thread of the workgroup calls it.
template <int NT>
SSA_TRI_INLINE void multisection_top(const double* D, const double* E2, int n, int k, double pivmin, double* lo,
                                     double* hi, double* xs, int* cnt, int rounds, int tid) {
    const int P = NT / k;  // shifts per eigenvalue per round
    const int ei = tid / P, p = tid % P;
    for (int round = 0; round < rounds; ++round) {
        if (ei < k) {
            const double a = lo[ei], b = hi[ei];
            const double x = a + (b - a) * (double)(p + 1) / (double)(P + 1);
            cnt[tid] = sturm_count(D, E2, n, x, pivmin);
            xs[tid] = x;
        }
        __syncthreads();
        if (ei < k && p == 0) {
            const int m = n - 1 - ei;  // the eigenvalue is the m-th smallest
            double a = lo[ei], b = hi[ei];
            for (int t = 0; t < P; ++t) {
                const int idx = ei * P + t;
                if (cnt[idx] <= m) {
                    a = xs[idx];
                } else {
                    b = xs[idx];
                    break;
                }
            }
            lo[ei] = a;
            hi[ei] = b;
        }
        __syncthreads();
    }
}

// Squared last component of the unit eigenvector of T_n at eigenvalue lam, from
// the twisted factorization of T - lam I (Dhillon and Parlett): backward pivots
// dm, forward pivots dp, twist index r minimizing |dp_r + dm_r - (D_r - lam)|,
// then z_r = 1 and z spreads both ways by products of pivot ratios, which keeps
// the tiny tail components of converged Ritz vectors to relative accuracy.
// dm and dp (n doubles each) live in the caller's scratch.
template <bool FAST = false>
SSA_TRI_INLINE double twisted_qlast(const double* D, const double* E2, int n, double lam, double pivmin, double* dm,
                                double* dp) {
    if (n == 1) return 1.0;
    dm[n - 1] = D[n - 1] - lam;
    for (int c = n - 2; c >= 0; --c) {
        const double x = fabs(dm[c + 1]) >= pivmin ? dm[c + 1] : -pivmin;
        dm[c] = D[c] - lam - tri_div<FAST>(E2[c], x);
    }
    double best = 0.0;
    int r = 0;
    for (int c = 0; c < n; ++c) {
        if (c == 0) {
            dp[0] = D[0] - lam;
        } else {
            const double x = fabs(dp[c - 1]) >= pivmin ? dp[c - 1] : -pivmin;
            dp[c] = D[c] - lam - tri_div<FAST>(E2[c - 1], x);
        }
        const double g = fabs(dp[c] + dm[c] - (D[c] - lam));
        if (c == 0 || g < best) {
            best = g;
            r = c;
        }
    }
    double z = 1.0, zz = 1.0;
    for (int c = r - 1; c >= 0; --c) {
        const double x = fabs(dp[c]) >= pivmin ? dp[c] : -pivmin;
        z = -tri_div<FAST>(sqrt(E2[c]), x) * z;
        zz += z * z;
    }
    z = 1.0;
    for (int c = r + 1; c < n; ++c) {
        const double x = fabs(dm[c]) >= pivmin ? dm[c] : -pivmin;
        z = -tri_div<FAST>(sqrt(E2[c - 1]), x) * z;
        zz += z * z;
    }
    const double zl = r == n - 1 ? 1.0 : z;
    return zl * zl / zz;
}

// Solve (T - lam I) x = x in place (partial pivoting; tiny pivots replaced).
template <bool FAST = false>
SSA_TRI_INLINE void shifted_solve(const double* D, const double* E, int n, double lam, double tnorm, double* x,
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
            const double f = tri_div<FAST>(cc[i], a[i]);
            a[i + 1] -= f * b[i];
            x[i + 1] -= f * x[i];
        } else {
            const double f = tri_div<FAST>(a[i], cc[i]);
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
    x[n - 1] = tri_div<FAST>(x[n - 1], a[n - 1]);
    if (n >= 2) x[n - 2] = tri_div<FAST>(x[n - 2] - b[n - 2] * x[n - 1], a[n - 2]);
    for (int i = n - 3; i >= 0; --i) x[i] = tri_div<FAST>(x[i] - b[i] * x[i + 1] - u2[i] * x[i + 2], a[i]);
}

}  // namespace ssa
