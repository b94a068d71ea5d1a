/*
 * ssa_oracle.c -- plain FP64 CPU oracle for Basic SSA (Korobeynikov,
 * "Computation- and Space-Efficient Implementation of SSA").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * (the HIP library) shares no code with it and never calls it.
 *
 * Everything here is written from the definitions in the paper, in double
 * precision, with no blocking, fusion or FFT:
 *   - embedding / trajectory matrix              (Sec. 2.1)
 *   - singular value decomposition               (Sec. 2.2), computed by a
 *     one-sided (Hestenes) Jacobi iteration on the explicit matrix, the
 *     method named in Sec. 3 as one that needs the matrix formed
 *   - diagonal averaging (Hankelization)         (Sec. 2.4, eq. hankelization)
 *   - rank-1 Hankelization as antidiagonal sums  (Sec. 5, eq. hankelization1)
 *   - grouping                                   (Sec. 2.3)
 * and for two-dimensional arrays (2D-SSA, named in Sec. 1 and Sec. 3.3 as the
 * case whose trajectory matrix is Hankel with Hankel blocks):
 *   - the 2D trajectory matrix, its SVD and the 2D diagonal averaging,
 *     from the definition (explicit matrix, the same Jacobi SVD, direct
 *     averaging over the index sets a + c = i, b + d = j);
 * and, for sizes where the explicit L x K matrix is too large ("tier B"):
 *   - Golub-Kahan-Lanczos bidiagonalization      (Sec. 3.1, Algorithm 1) with
 *     full reorthogonalization by modified Gram-Schmidt applied twice
 *     (Sec. 3.2.2), where every product X v and X^T u is evaluated row by
 *     row from the series itself (X never stored, no FFT), followed by the
 *     same Jacobi SVD of the small bidiagonal matrix B_j and the Ritz
 *     extraction implied by eqs. lbdiagm1/lbdiagm2.
 *
 * Index convention: 0-based.  Series f[0..N-1], K = N - L + 1,
 * X[i][j] = f[i + j] for 0 <= i < L, 0 <= j < K.
 *
 * Conventions of the exported functions: all arrays are host memory owned
 * by the caller; matrices are row-major unless stated; a negative return
 * value means invalid arguments, 0 success, a positive value a warning.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double dot(const double* a, const double* b, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sec. 2.1: the L-trajectory matrix, X[i][j] = f[i+j] (row-major L x K). */
int oracle_trajectory(const double* f, long N, long L, double* X) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
    for (long i = 0; i < L; ++i)
        for (long j = 0; j < K; ++j) X[i * K + j] = f[i + j];
    return 0;
}

/*
 * One-sided Jacobi SVD of a dense m x n matrix A (row-major, overwritten).
 * Let r = min(m, n).  Outputs: sigma[r] descending, U (m x r row-major),
 * V (n x r row-major) with A = U diag(sigma) V^T.  Columns belonging to a
 * zero singular value are returned as zero vectors (the null space is not
 * unique, so it is not reported).
 *
 * Method: with m <= n the m rows of A are made mutually orthogonal by plane
 * rotations (Hestenes); the rotations accumulate into an m x m orthogonal
 * J so that J^T A has orthogonal rows.  Then sigma_p = |row p|,
 * v_p = row p / sigma_p and u_p = column p of J.  A pair (p, q) is rotated
 * when |<a_p, a_q>| > tol * |a_p| |a_q|; the sweep order is the fixed
 * cyclic row order.  If m > n the transpose is decomposed and U, V swap.
 * Returns the number of sweeps, or -2 if max_sweeps was exhausted.
 */
static int jacobi_rows(double* A, long m, long n, double tol, int max_sweeps,
                       double* J /* m x m, row-major, J[:,p] stored as row p of Jt */) {
    /* Jt[p*m + i] = J[i][p] */
    double* Jt = J;
    for (long p = 0; p < m; ++p)
        for (long i = 0; i < m; ++i) Jt[p * m + i] = (p == i) ? 1.0 : 0.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (long p = 0; p < m - 1; ++p) {
            for (long q = p + 1; q < m; ++q) {
                double* ap = A + p * n;
                double* aq = A + q * n;
                double a = dot(ap, ap, n);
                double b = dot(aq, aq, n);
                double c = dot(ap, aq, n);
                if (a == 0.0 || b == 0.0) continue;
                if (fabs(c) <= tol * sqrt(a) * sqrt(b)) continue;
                rotated = 1;
                double zeta = (b - a) / (2.0 * c);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (long i = 0; i < n; ++i) {
                    double xp = ap[i], xq = aq[i];
                    ap[i] = cs * xp - sn * xq;
                    aq[i] = sn * xp + cs * xq;
                }
                double* jp = Jt + p * m;
                double* jq = Jt + q * m;
                for (long i = 0; i < m; ++i) {
                    double xp = jp[i], xq = jq[i];
                    jp[i] = cs * xp - sn * xq;
                    jq[i] = sn * xp + cs * xq;
                }
            }
        }
        if (!rotated) return sweep;
    }
    return -2;
}

int oracle_jacobi_svd(const double* A_in, long m, long n, double tol, int max_sweeps,
                      double* sigma, double* U, double* V) {
    if (m <= 0 || n <= 0) return -1;
    int transposed = m > n;
    long mm = transposed ? n : m; /* number of rows rotated */
    long nn = transposed ? m : n;
    double* A = (double*)malloc(sizeof(double) * mm * nn);
    double* Jt = (double*)malloc(sizeof(double) * mm * mm);
    long* order = (long*)malloc(sizeof(long) * mm);
    double* s = (double*)malloc(sizeof(double) * mm);
    if (!A || !Jt || !order || !s) { free(A); free(Jt); free(order); free(s); return -3; }
    if (!transposed) {
        memcpy(A, A_in, sizeof(double) * m * n);
    } else {
        for (long i = 0; i < m; ++i)
            for (long j = 0; j < n; ++j) A[j * m + i] = A_in[i * n + j];
    }
    int sweeps = jacobi_rows(A, mm, nn, tol, max_sweeps, Jt);
    for (long p = 0; p < mm; ++p) {
        s[p] = sqrt(dot(A + p * nn, A + p * nn, nn));
        order[p] = p;
    }
    /* sort descending by sigma (insertion sort: r is small) */
    for (long a = 1; a < mm; ++a) {
        long key = order[a];
        long b = a - 1;
        while (b >= 0 && s[order[b]] < s[key]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = key;
    }
    /* rows-side vectors: columns of J (length mm); other side: normalized rows (length nn) */
    double* Rside = transposed ? V : U; /* mm x mm */
    double* Cside = transposed ? U : V; /* nn x mm */
    for (long c = 0; c < mm; ++c) {
        long p = order[c];
        sigma[c] = s[p];
        for (long i = 0; i < mm; ++i) Rside[i * mm + c] = Jt[p * mm + i];
        double inv = s[p] > 0.0 ? 1.0 / s[p] : 0.0;
        for (long i = 0; i < nn; ++i) Cside[i * mm + c] = A[p * nn + i] * inv;
    }
    free(A); free(Jt); free(order); free(s);
    return sweeps;
}

/* Sec. 2.4 (eq. hankelization): diagonal averaging of a general L x K matrix Y. */
int oracle_hankelize(const double* Y, long L, long K, double* g) {
    if (L <= 0 || K <= 0) return -1;
    long N = L + K - 1;
    for (long n = 0; n < N; ++n) {
        double s = 0.0;
        long cnt = 0;
        for (long i = 0; i < L; ++i) {
            long j = n - i;
            if (j < 0 || j >= K) continue;
            s += Y[i * K + j];
            ++cnt;
        }
        g[n] = s / (double)cnt;
    }
    return 0;
}

/* Sec. 5 (eq. hankelization1): diagonal averaging of sigma * u v^T. */
int oracle_rank1_hankelize(double sigma, const double* u, long L, const double* v, long K,
                           double* g) {
    if (L <= 0 || K <= 0) return -1;
    long N = L + K - 1;
    for (long n = 0; n < N; ++n) {
        double s = 0.0;
        long cnt = 0;
        for (long i = 0; i < L; ++i) {
            long j = n - i;
            if (j < 0 || j >= K) continue;
            s += u[i] * v[j];
            ++cnt;
        }
        g[n] = sigma * s / (double)cnt;
    }
    return 0;
}

/*
 * Sec. 2.3 + 2.4: for each group I_g (CSR: offsets[m+1], members[] are
 * 0-based triple indices), out[g*N + n] = Hankelization of sum_{i in I_g}
 * sigma_i u_i v_i^T.  U is L x k row-major, V is K x k row-major.
 */
int oracle_reconstruct(long N, long L, int k, const double* sigma, const double* U,
                       const double* V, const int* offsets, const int* members, int m,
                       double* out) {
    if (N <= 2 || L <= 1 || L >= N || k <= 0 || m <= 0) return -1;
    long K = N - L + 1;
    double* u = (double*)malloc(sizeof(double) * L);
    double* v = (double*)malloc(sizeof(double) * K);
    double* g = (double*)malloc(sizeof(double) * N);
    if (!u || !v || !g) { free(u); free(v); free(g); return -3; }
    for (int grp = 0; grp < m; ++grp) {
        double* o = out + (long)grp * N;
        for (long n = 0; n < N; ++n) o[n] = 0.0;
        for (int t = offsets[grp]; t < offsets[grp + 1]; ++t) {
            int i = members[t];
            if (i < 0 || i >= k) { free(u); free(v); free(g); return -1; }
            for (long a = 0; a < L; ++a) u[a] = U[a * k + i];
            for (long b = 0; b < K; ++b) v[b] = V[b * k + i];
            oracle_rank1_hankelize(sigma[i], u, L, v, K, g);
            for (long n = 0; n < N; ++n) o[n] += g[n];
        }
    }
    free(u); free(v); free(g);
    return 0;
}

/*
 * Tier A: truncated SVD from the definition (Sec. 2.1-2.2).  Forms X,
 * computes its full Jacobi SVD and returns the k leading triples:
 * sigma[k], U (L x k row-major), V (K x k row-major).
 */
int oracle_ssa_dense(const double* f, long N, long L, int k, double* sigma, double* U,
                     double* V) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
    long r = L < K ? L : K;
    if (k < 1 || k > r) return -1;
    double* X = (double*)malloc(sizeof(double) * L * K);
    double* s = (double*)malloc(sizeof(double) * r);
    double* UU = (double*)malloc(sizeof(double) * L * r);
    double* VV = (double*)malloc(sizeof(double) * K * r);
    if (!X || !s || !UU || !VV) { free(X); free(s); free(UU); free(VV); return -3; }
    oracle_trajectory(f, N, L, X);
    int sweeps = oracle_jacobi_svd(X, L, K, 1e-15, 60, s, UU, VV);
    for (int c = 0; c < k; ++c) sigma[c] = s[c];
    for (long i = 0; i < L; ++i)
        for (int c = 0; c < k; ++c) U[i * k + c] = UU[i * r + c];
    for (long i = 0; i < K; ++i)
        for (int c = 0; c < k; ++c) V[i * k + c] = VV[i * r + c];
    free(X); free(s); free(UU); free(VV);
    return sweeps < 0 ? 1 : 0;
}

/* (X v)[i] = sum_j f[i+j] v[j], i < L: one row of the trajectory matrix at a time. */
int oracle_matvec(const double* f, long N, long L, const double* v, double* out) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < L; ++i) out[i] = dot(f + i, v, K);
    return 0;
}

/* (X^T u)[j] = sum_i f[i+j] u[i], j < K: one column of the trajectory matrix at a time. */
int oracle_rmatvec(const double* f, long N, long L, const double* u, double* out) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < K; ++j) out[j] = dot(f + j, u, L);
    return 0;
}

/* Selected entries of a product with the trajectory matrix (Sec. 2.1), for
 * sizes where a whole product is too slow ("tier C" certificates):
 *   transpose = 0: out[q] = (X x)[rows[q]]   = sum_j f[rows[q] + j] x[j], x of length K;
 *   transpose = 1: out[q] = (X^T x)[rows[q]] = sum_i f[i + rows[q]] x[i], x of length L.
 * Each entry is the plain dot product of one row (column) of X with x. */
int oracle_matvec_rows(const double* f, long N, long L, int transpose, const double* x,
                       const long* rows, long nrows, double* out) {
    if (N <= 2 || L <= 1 || L >= N || nrows < 0) return -1;
    long K = N - L + 1;
    long lim = transpose ? K : L, len = transpose ? L : K;
    for (long q = 0; q < nrows; ++q)
        if (rows[q] < 0 || rows[q] >= lim) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < nrows; ++q) out[q] = dot(f + rows[q], x, len);
    return 0;
}

/* Sec. 2.4 (eq. hankelization) at selected positions only: the mean of
 * sigma * u[a] * v[b] over the antidiagonal a + b = n of sigma u v^T, for each
 * n = pos[q] (0 <= n < L + K - 1). */
int oracle_hankelize_at(double sigma, const double* u, long L, const double* v, long K,
                        const long* pos, long npos, double* out) {
    if (L <= 0 || K <= 0 || npos < 0) return -1;
    for (long q = 0; q < npos; ++q)
        if (pos[q] < 0 || pos[q] >= L + K - 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < npos; ++q) {
        long n = pos[q];
        long a0 = n - (K - 1) > 0 ? n - (K - 1) : 0, a1 = n < L - 1 ? n : L - 1;
        double acc = 0.0;
        for (long a = a0; a <= a1; ++a) acc += u[a] * v[n - a];
        out[q] = sigma * acc / (double)(a1 - a0 + 1);
    }
    return 0;
}

/*
 * Structural-change detection (Sec. "Detection of Structural Changes", eq. g):
 * the heterogeneity index of a test series F2 against a base series F1 is
 *   g = sum_j dist^2(X2_j, span{U1_i, i in I}) / sum_j |X2_j|^2,
 * over the L-lagged vectors X2_j of F2 (j < T - L + 1), with U1_i the
 * eigenvectors of the trajectory matrix of F1 (window L).  The H-matrix holds
 * g for base windows f[i .. i+B-1] and test windows f[j .. j+T-1] (0-based
 * starts i < N-B+1, j < N-T+1), row-major, G[i * (N-T+1) + j].  I holds
 * 1-based triple indices.  A test window with no energy gets g = 0.
 * Each dist^2 is ||X - sum_i (U_i^T X) U_i||^2 evaluated as written.
 */
int oracle_hmatrix(const double* f, long N, long B, long T, long L, const int* I, int nI, double* G) {
    if (nI < 1 || B > N || T > N || L <= 1 || L >= B - 1 || L > T) return -1;
    int k = 0;
    for (int q = 0; q < nI; ++q) {
        if (I[q] < 1 || I[q] > L) return -1;
        if (I[q] > k) k = I[q];
    }
    const long MB = N - B + 1, MT = N - T + 1, K2 = T - L + 1;
    if (k > (B - L + 1 < L ? B - L + 1 : L)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < MB; ++i) {
        double* sg = (double*)malloc(sizeof(double) * k);
        double* U = (double*)malloc(sizeof(double) * L * k);
        double* V = (double*)malloc(sizeof(double) * (B - L + 1) * k);
        double* x = (double*)malloc(sizeof(double) * L);
        if (!sg || !U || !V || !x || oracle_ssa_dense(f + i, B, L, k, sg, U, V) < 0) {
#pragma omp atomic write
            bad = 1;
        } else {
            for (long j = 0; j < MT; ++j) {
                double num = 0.0, den = 0.0;
                for (long m = 0; m < K2; ++m) {
                    const double* X = f + j + m;  /* lagged vector m of the test window */
                    for (long l = 0; l < L; ++l) x[l] = X[l];
                    for (int q = 0; q < nI; ++q) {
                        const int c = I[q] - 1;
                        double p = 0.0;
                        for (long l = 0; l < L; ++l) p += U[l * k + c] * X[l];
                        for (long l = 0; l < L; ++l) x[l] -= p * U[l * k + c];
                    }
                    for (long l = 0; l < L; ++l) {
                        num += x[l] * x[l];
                        den += X[l] * X[l];
                    }
                }
                G[i * MT + j] = den > 0.0 ? num / den : 0.0;
            }
        }
        free(sg); free(U); free(V); free(x);
    }
    return bad ? -3 : 0;
}

/*
 * Repeated realizations (Sec. "Bootstrap Confidence Intervals Construction"):
 * each of the R series F_r (row r of F_all, N values) is reconstructed from
 * its first d eigentriples (window L, Sec. 2.3-2.4 with the group {1..d}),
 * G_r; then per point n
 *   mean[n] = (1/R) sum_r G_r[n],
 *   var[n]  = (1/(R-1)) sum_r (G_r[n] - mean[n])^2   (0 when R = 1),
 *   mse[n]  = (1/R) sum_r (G_r[n] - truth[n])^2      (if truth and mse are given).
 */
int oracle_realization_stats(const double* F_all, long R, long N, long L, int d, const double* truth,
                             double* mean, double* var, double* mse) {
    if (R < 1 || N <= 2 || L <= 1 || L >= N || d < 1) return -1;
    const long K = N - L + 1;
    if (d > (L < K ? L : K)) return -1;
    double* G = (double*)malloc(sizeof(double) * R * N);
    if (!G) return -3;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < R; ++r) {
        double* sg = (double*)malloc(sizeof(double) * d);
        double* U = (double*)malloc(sizeof(double) * L * d);
        double* V = (double*)malloc(sizeof(double) * K * d);
        int offs[2] = {0, d};
        int* mem = (int*)malloc(sizeof(int) * d);
        if (!sg || !U || !V || !mem || oracle_ssa_dense(F_all + r * N, N, L, d, sg, U, V) < 0) {
#pragma omp atomic write
            bad = 1;
        } else {
            for (int c = 0; c < d; ++c) mem[c] = c;
            if (oracle_reconstruct(N, L, d, sg, U, V, offs, mem, 1, G + r * N) < 0) {
#pragma omp atomic write
                bad = 1;
            }
        }
        free(sg); free(U); free(V); free(mem);
    }
    if (!bad) {
        for (long n = 0; n < N; ++n) {
            double m = 0.0;
            for (long r = 0; r < R; ++r) m += G[r * N + n];
            m /= (double)R;
            double v = 0.0, e = 0.0;
            for (long r = 0; r < R; ++r) {
                const double x = G[r * N + n];
                v += (x - m) * (x - m);
                if (truth) e += (x - truth[n]) * (x - truth[n]);
            }
            mean[n] = m;
            var[n] = R > 1 ? v / (double)(R - 1) : 0.0;
            if (truth && mse) mse[n] = e / (double)R;
        }
    }
    free(G);
    return bad ? -3 : 0;
}

/* Modified Gram-Schmidt of x (length n) against ncol orthonormal columns
 * stored contiguously in Q (column c at Q + c*n). */
static void mgs(double* x, const double* Q, long ncol, long n) {
    for (long c = 0; c < ncol; ++c) {
        const double* q = Q + c * n;
        double h = dot(q, x, n);
        for (long i = 0; i < n; ++i) x[i] -= h * q[i];
    }
}

/*
 * Tier B: Golub-Kahan-Lanczos bidiagonalization (Algorithm 1) with full
 * reorthogonalization (MGS, applied twice, against all previous vectors),
 * matrix-vector products evaluated directly from the series.
 *
 * Inputs:  f[N], L, k, d_max (Krylov dimension cap), p0[L] (start vector),
 *          restart[n_restart * max(L,K)] (replacement directions used when a
 *          recurrence coefficient vanishes), check_every, tol.
 * Outputs: sigma[k], U (L x k row-major), V (K x k row-major), *steps.
 * Stopping: after step j (with alpha_{j+1} computed), the Jacobi SVD of the
 * (j+1) x j bidiagonal B_j = P diag(w) Q^T gives Ritz values w_i and, from
 * A^T U_{j+1} = V_j B_j^T + alpha_{j+1} v_{j+1} e_{j+1}^T, the residual
 * alpha_{j+1} |P[j][i]|.  Stop when every residual of the k leading values is
 * <= tol * w_1 and those values moved by less than tol relative to the
 * previous check.  Returns 0 converged, 1 if d_max was reached first.
 */
int oracle_lanczos_svd(const double* f, long N, long L, int k, int d_max, const double* p0,
                       const double* restart, int n_restart, int check_every, double tol,
                       double* sigma, double* U, double* V, int* steps) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
    long r = L < K ? L : K;
    if (k < 1 || k > r || d_max < k) return -1;
    if (d_max > r) d_max = (int)r;
    long nmax = L > K ? L : K;
    double* Ub = (double*)calloc((size_t)(d_max + 1) * L, sizeof(double));
    double* Vb = (double*)calloc((size_t)(d_max + 1) * K, sizeof(double));
    double* alpha = (double*)calloc((size_t)d_max + 2, sizeof(double));
    double* beta = (double*)calloc((size_t)d_max + 2, sizeof(double));
    double* x = (double*)malloc(sizeof(double) * nmax);
    double* B = (double*)malloc(sizeof(double) * (size_t)(d_max + 1) * d_max);
    double* w = (double*)malloc(sizeof(double) * d_max);
    double* P = (double*)malloc(sizeof(double) * (size_t)(d_max + 1) * d_max);
    double* Q = (double*)malloc(sizeof(double) * (size_t)d_max * d_max);
    double* wprev = (double*)malloc(sizeof(double) * k);
    if (!Ub || !Vb || !alpha || !beta || !x || !B || !w || !P || !Q || !wprev) {
        free(Ub); free(Vb); free(alpha); free(beta); free(x); free(B); free(w); free(P);
        free(Q); free(wprev);
        return -3;
    }
    int used_restart = 0;
    double bnorm = 0.0;
    /* u_1 = p0 / |p0|, beta_1 = |p0| */
    double nrm = sqrt(dot(p0, p0, L));
    for (long i = 0; i < L; ++i) Ub[i] = p0[i] / nrm;
    beta[1] = nrm;
    int have_prev = 0, converged = 0, jdone = 0;
    for (int j = 1; j <= d_max; ++j) {
        /* r_j = X^T u_j - beta_j v_{j-1} */
        oracle_rmatvec(f, N, L, Ub + (long)(j - 1) * L, x);
        if (j > 1)
            for (long i = 0; i < K; ++i) x[i] -= beta[j] * Vb[(long)(j - 2) * K + i];
        mgs(x, Vb, j - 1, K);
        mgs(x, Vb, j - 1, K);
        double a = sqrt(dot(x, x, K));
        if (a <= 1e-13 * (bnorm > 0.0 ? bnorm : 1.0)) {
            /* alpha_j vanishes: record zero and continue from a fresh direction */
            a = 0.0;
            if (used_restart >= n_restart) { jdone = j - 1; break; }
            memcpy(x, restart + (long)used_restart * nmax, sizeof(double) * K);
            ++used_restart;
            mgs(x, Vb, j - 1, K);
            mgs(x, Vb, j - 1, K);
            double s = sqrt(dot(x, x, K));
            for (long i = 0; i < K; ++i) x[i] /= s;
        } else {
            for (long i = 0; i < K; ++i) x[i] /= a;
        }
        alpha[j] = a;
        if (a > bnorm) bnorm = a;
        memcpy(Vb + (long)(j - 1) * K, x, sizeof(double) * K);

        /* convergence test on B_{j-1} now that alpha_j is known */
        if (j - 1 >= k && ((j - 1) % check_every == 0)) {
            int jj = j - 1;
            for (long t = 0; t < (long)(jj + 1) * jj; ++t) B[t] = 0.0;
            for (int c = 0; c < jj; ++c) {
                B[(long)c * jj + c] = alpha[c + 1];
                B[(long)(c + 1) * jj + c] = beta[c + 2];
            }
            oracle_jacobi_svd(B, jj + 1, jj, 1e-15, 80, w, P, Q);
            int ok = have_prev;
            for (int i = 0; i < k; ++i) {
                double res = alpha[j] * fabs(P[(long)jj * jj + i]);
                if (res > tol * w[0]) ok = 0;
                if (have_prev && fabs(w[i] - wprev[i]) > tol * w[0]) ok = 0;
            }
            for (int i = 0; i < k; ++i) wprev[i] = w[i];
            have_prev = 1;
            if (ok) { converged = 1; jdone = jj; break; }
        }

        /* p_j = X v_j - alpha_j u_j */
        oracle_matvec(f, N, L, Vb + (long)(j - 1) * K, x);
        for (long i = 0; i < L; ++i) x[i] -= alpha[j] * Ub[(long)(j - 1) * L + i];
        mgs(x, Ub, j, L);
        mgs(x, Ub, j, L);
        double b = sqrt(dot(x, x, L));
        if (b <= 1e-13 * (bnorm > 0.0 ? bnorm : 1.0) || j == r) {
            b = 0.0;
            if (j == r || used_restart >= n_restart) {
                beta[j + 1] = 0.0;
                jdone = j;
                if (j == r) converged = 1;
                break;
            }
            memcpy(x, restart + (long)used_restart * nmax, sizeof(double) * L);
            ++used_restart;
            mgs(x, Ub, j, L);
            mgs(x, Ub, j, L);
            double s = sqrt(dot(x, x, L));
            for (long i = 0; i < L; ++i) x[i] /= s;
        } else {
            for (long i = 0; i < L; ++i) x[i] /= b;
        }
        beta[j + 1] = b;
        if (b > bnorm) bnorm = b;
        memcpy(Ub + (long)j * L, x, sizeof(double) * L);
        jdone = j;
    }
    int jj = jdone;
    /* final SVD of B_jj and Ritz vectors U_{jj+1} P, V_jj Q */
    for (long t = 0; t < (long)(jj + 1) * jj; ++t) B[t] = 0.0;
    for (int c = 0; c < jj; ++c) {
        B[(long)c * jj + c] = alpha[c + 1];
        B[(long)(c + 1) * jj + c] = beta[c + 2];
    }
    oracle_jacobi_svd(B, jj + 1, jj, 1e-15, 80, w, P, Q);
    int kk = k < jj ? k : jj;
    for (int i = 0; i < k; ++i) sigma[i] = i < kk ? w[i] : 0.0;
    for (long a = 0; a < L; ++a)
        for (int i = 0; i < k; ++i) {
            double s = 0.0;
            if (i < kk)
                for (int c = 0; c <= jj; ++c) s += Ub[(long)c * L + a] * P[(long)c * jj + i];
            U[a * k + i] = s;
        }
    for (long b2 = 0; b2 < K; ++b2)
        for (int i = 0; i < k; ++i) {
            double s = 0.0;
            if (i < kk)
                for (int c = 0; c < jj; ++c) s += Vb[(long)c * K + b2] * Q[(long)c * jj + i];
            V[b2 * k + i] = s;
        }
    if (steps) *steps = jj;
    free(Ub); free(Vb); free(alpha); free(beta); free(x); free(B); free(w); free(P);
    free(Q); free(wprev);
    return converged ? 0 : 1;
}

/*
 * Raw Golub-Kahan-Lanczos run (Algorithm 1 with MGS-twice reorthogonalization)
 * for exactly d steps, returning the bases and the bidiagonal so that tests can
 * check the relations X V_d = U_{d+1} B_d and X^T U_{d+1} = V_d B_d^T +
 * alpha_{d+1} v_{d+1} e^T (eqs. lbdiagm1 / lbdiagm2).  Ub: (d+1) x L (row c =
 * u_{c+1}), Vb: (d+1) x K, alpha[d+2], beta[d+2] (1-based as in the paper).
 */
int oracle_gkl_raw(const double* f, long N, long L, int d, const double* p0, double* Ub,
                   double* Vb, double* alpha, double* beta) {
    if (N <= 2 || L <= 1 || L >= N) return -1;
    long K = N - L + 1;
    long r = L < K ? L : K;
    if (d < 1 || d >= r) return -1;
    long nmax = L > K ? L : K;
    double* x = (double*)malloc(sizeof(double) * nmax);
    if (!x) return -3;
    for (int t = 0; t < d + 2; ++t) { alpha[t] = 0.0; beta[t] = 0.0; }
    double nrm = sqrt(dot(p0, p0, L));
    for (long i = 0; i < L; ++i) Ub[i] = p0[i] / nrm;
    beta[1] = nrm;
    for (int j = 1; j <= d + 1; ++j) {
        oracle_rmatvec(f, N, L, Ub + (long)(j - 1) * L, x);
        if (j > 1)
            for (long i = 0; i < K; ++i) x[i] -= beta[j] * Vb[(long)(j - 2) * K + i];
        mgs(x, Vb, j - 1, K);
        mgs(x, Vb, j - 1, K);
        double a = sqrt(dot(x, x, K));
        alpha[j] = a;
        for (long i = 0; i < K; ++i) Vb[(long)(j - 1) * K + i] = x[i] / a;
        if (j == d + 1) break;
        oracle_matvec(f, N, L, Vb + (long)(j - 1) * K, x);
        for (long i = 0; i < L; ++i) x[i] -= a * Ub[(long)(j - 1) * L + i];
        mgs(x, Ub, j, L);
        mgs(x, Ub, j, L);
        double b = sqrt(dot(x, x, L));
        beta[j + 1] = b;
        for (long i = 0; i < L; ++i) Ub[(long)j * L + i] = x[i] / b;
    }
    free(x);
    return 0;
}

/*
 * 2D-SSA.  An Nx x Ny array F (row-major, F[i][j] at i * Ny + j) with window
 * Lx x Ly; Kx = Nx - Lx + 1, Ky = Ny - Ly + 1.  Each column of the trajectory
 * matrix is one Lx x Ly sub-array of F, read row by row:
 *   X[(a, b), (c, d)] = F[a + c][b + d],
 * row index a * Ly + b (a < Lx, b < Ly), column index c * Ky + d (c < Kx,
 * d < Ky); X is (Lx Ly) x (Kx Ky), Hankel with Hankel blocks.
 */
static int check_2d(long Nx, long Ny, long Lx, long Ly) {
    if (Nx < 1 || Ny < 1 || Lx < 1 || Ly < 1 || Lx > Nx || Ly > Ny) return -1;
    if (Lx * Ly < 2 || (Nx - Lx + 1) * (Ny - Ly + 1) < 2) return -1;
    return 0;
}

int oracle_trajectory_2d(const double* F, long Nx, long Ny, long Lx, long Ly, double* X) {
    if (check_2d(Nx, Ny, Lx, Ly)) return -1;
    long Kx = Nx - Lx + 1, Ky = Ny - Ly + 1, ncol = Kx * Ky;
    for (long a = 0; a < Lx; ++a)
        for (long b = 0; b < Ly; ++b)
            for (long c = 0; c < Kx; ++c)
                for (long d = 0; d < Ky; ++d)
                    X[(a * Ly + b) * ncol + c * Ky + d] = F[(a + c) * Ny + (b + d)];
    return 0;
}

/*
 * 2D diagonal averaging of an (Lx Ly) x (Kx Ky) matrix Y: G[i][j] is the
 * mean of Y[(a, b), (c, d)] over all a + c = i, b + d = j (G is Nx x Ny).
 */
int oracle_hankelize_2d(const double* Y, long Nx, long Ny, long Lx, long Ly, double* G) {
    if (check_2d(Nx, Ny, Lx, Ly)) return -1;
    long Kx = Nx - Lx + 1, Ky = Ny - Ly + 1, ncol = Kx * Ky;
    for (long i = 0; i < Nx; ++i)
        for (long j = 0; j < Ny; ++j) {
            double s = 0.0;
            long cnt = 0;
            for (long a = 0; a < Lx; ++a) {
                long c = i - a;
                if (c < 0 || c >= Kx) continue;
                for (long b = 0; b < Ly; ++b) {
                    long d = j - b;
                    if (d < 0 || d >= Ky) continue;
                    s += Y[(a * Ly + b) * ncol + c * Ky + d];
                    ++cnt;
                }
            }
            G[i * Ny + j] = s / (double)cnt;
        }
    return 0;
}

/*
 * 2D-SSA from the definition: the k leading triples of the explicit 2D
 * trajectory matrix (Jacobi SVD): sigma[k], U ((Lx Ly) x k row-major; column
 * i reshaped row by row is the Lx x Ly eigen-array), V ((Kx Ky) x k).
 */
int oracle_ssa2d_dense(const double* F, long Nx, long Ny, long Lx, long Ly, int k, double* sigma,
                       double* U, double* V) {
    if (check_2d(Nx, Ny, Lx, Ly)) return -1;
    long L = Lx * Ly, K = (Nx - Lx + 1) * (Ny - Ly + 1);
    long r = L < K ? L : K;
    if (k < 1 || k > r) return -1;
    double* X = (double*)malloc(sizeof(double) * L * K);
    double* s = (double*)malloc(sizeof(double) * r);
    double* UU = (double*)malloc(sizeof(double) * L * r);
    double* VV = (double*)malloc(sizeof(double) * K * r);
    if (!X || !s || !UU || !VV) { free(X); free(s); free(UU); free(VV); return -3; }
    oracle_trajectory_2d(F, Nx, Ny, Lx, Ly, X);
    int sweeps = oracle_jacobi_svd(X, L, K, 1e-15, 60, s, UU, VV);
    for (int c = 0; c < k; ++c) sigma[c] = s[c];
    for (long i = 0; i < L; ++i)
        for (int c = 0; c < k; ++c) U[i * k + c] = UU[i * r + c];
    for (long i = 0; i < K; ++i)
        for (int c = 0; c < k; ++c) V[i * k + c] = VV[i * r + c];
    free(X); free(s); free(UU); free(VV);
    return sweeps < 0 ? 1 : 0;
}

/*
 * Grouping + 2D diagonal averaging: out[g] (Nx x Ny) is the 2D averaging of
 * sum_{i in I_g} sigma_i U_i V_i^T, each term averaged directly:
 * G[i][j] = sigma / cnt * sum_{a + c = i, b + d = j} U[(a, b)] V[(c, d)].
 */
int oracle_reconstruct_2d(long Nx, long Ny, long Lx, long Ly, int k, const double* sigma,
                          const double* U, const double* V, const int* offsets, const int* members,
                          int m, double* out) {
    if (check_2d(Nx, Ny, Lx, Ly) || k <= 0 || m <= 0) return -1;
    long Kx = Nx - Lx + 1, Ky = Ny - Ly + 1;
    for (int grp = 0; grp < m; ++grp) {
        for (int t = offsets[grp]; t < offsets[grp + 1]; ++t)
            if (members[t] < 0 || members[t] >= k) return -1;
        double* o = out + (long)grp * Nx * Ny;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < Nx; ++i)
            for (long j = 0; j < Ny; ++j) {
                double acc = 0.0;
                long cnt = 0;
                for (long a = 0; a < Lx; ++a) {
                    long c = i - a;
                    if (c < 0 || c >= Kx) continue;
                    for (long b = 0; b < Ly; ++b) {
                        long d = j - b;
                        if (d < 0 || d >= Ky) continue;
                        ++cnt;
                        for (int t = offsets[grp]; t < offsets[grp + 1]; ++t) {
                            int q = members[t];
                            acc += sigma[q] * U[(a * Ly + b) * k + q] * V[(c * Ky + d) * k + q];
                        }
                    }
                }
                o[i * Ny + j] = acc / (double)cnt;
            }
    }
    return 0;
}
