// small_svd.cpp -- Ritz values and vectors of the Lanczos bidiagonal B_d.
//
// After d steps of Algorithm 1, B_d is (d+1) x d lower bidiagonal with alpha_j
// on the diagonal and beta_{j+1} below it (Sec. 3.1).  Its singular triples
// (omega_i, p_i, q_i) give the Ritz approximations omega_i, U_{d+1} p_i,
// V_d q_i, and the relation X^T U_{d+1} = V_d B_d^T + alpha_{d+1} v_{d+1}
// e_{d+1}^T (eq. lbdiagm2) bounds their residual by alpha_{d+1} |p_i[d]|.
//
// The right singular vectors of B_d are the eigenvectors of the symmetric
// tridiagonal T = B_d^T B_d (the cross-product route of Theorem 1), with
//   T[c][c] = alpha_{c+1}^2 + beta_{c+2}^2,  T[c][c+1] = alpha_{c+2} beta_{c+2}.
// Eigenvalues come from the implicit QL iteration with Wilkinson shifts
// (Bowdler, Martin, Reinsch and Wilkinson 1968), O(d^2); while iterating only
// the last row of the eigenvector matrix is carried, which is all the
// residual bound needs: p_i[d] = beta_{d+1} q_i[d-1] / omega_i.  The final k
// vectors come from inverse iteration on T (Wilkinson), each made orthogonal
// to the ones before it, O(k^2 d).  The left vectors are p_i = B_d q_i / omega_i,
// made orthogonal to the earlier ones; where omega_i = 0 (a series of rank below k)
// a unit vector orthogonal to them takes its place, so P stays orthonormal.
//
// Squaring costs relative accuracy only for omega_i below ~1e-8 omega_1, far
// under the error of the FP32 products that produced B_d.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ssa_internal.h"

namespace ssa {

namespace {

constexpr double kEps = 2.220446049250313e-16;

void form_tridiagonal(const double* alpha, const double* beta, int d, double* D, double* E) {
    for (int c = 0; c < d; ++c) D[c] = alpha[c + 1] * alpha[c + 1] + beta[c + 2] * beta[c + 2];
    for (int c = 0; c + 1 < d; ++c) E[c] = alpha[c + 2] * beta[c + 2];
    E[d - 1] = 0.0;
}

// Implicit QL with shifts on the symmetric tridiagonal (D diagonal, E[c]
// couples c and c+1).  D receives the eigenvalues (unordered).  If zl is
// given (initialized to the last row of the identity) the same rotations are
// applied to it, so on exit zl[c] is the last component of the eigenvector
// of D[c].  Returns false if an eigenvalue needed more than 64 iterations.
bool tridiag_ql(int n, double* D, double* E, double* zl) {
    if (n <= 0) return true;
    E[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(D[m]) + std::fabs(D[m + 1]);
                if (std::fabs(E[m]) <= kEps * dd) break;
            }
            if (m == l) break;
            if (++iter > 64) return false;
            // shift from the leading 2x2 block of the unreduced part
            double g = (D[l + 1] - D[l]) / (2.0 * E[l]);
            double r = std::hypot(g, 1.0);
            g = D[m] - D[l] + E[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool underflow = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * E[i];
                const double b = c * E[i];
                r = std::hypot(f, g);
                E[i + 1] = r;
                if (r == 0.0) {
                    D[i + 1] -= p;
                    E[m] = 0.0;
                    underflow = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = D[i + 1] - p;
                r = (D[i] - g) * s + 2.0 * c * b;
                p = s * r;
                D[i + 1] = g + p;
                g = c * r - b;
                if (zl) {
                    const double z1 = zl[i + 1];
                    zl[i + 1] = s * zl[i] + c * z1;
                    zl[i] = c * zl[i] - s * z1;
                }
            }
            if (underflow) continue;
            D[l] -= p;
            E[l] = g;
            E[m] = 0.0;
        }
    }
    return true;
}

// Solve (T - lam I) x = rhs (in place in rhs) by Gaussian elimination with
// partial pivoting on the tridiagonal; tiny pivots are replaced by
// eps * tnorm (the usual inverse-iteration safeguard).
void shifted_solve(int n, const double* D, const double* E, double lam, double tnorm, double* rhs,
                   double* a, double* b, double* c, double* u2) {
    for (int i = 0; i < n; ++i) a[i] = D[i] - lam;
    for (int i = 0; i + 1 < n; ++i) {
        b[i] = E[i];
        c[i] = E[i];
    }
    const double tiny = kEps * (tnorm > 0.0 ? tnorm : 1.0);
    for (int i = 0; i + 1 < n; ++i) {
        u2[i] = 0.0;
        if (std::fabs(a[i]) >= std::fabs(c[i])) {
            if (a[i] == 0.0) a[i] = tiny;
            const double f = c[i] / a[i];
            a[i + 1] -= f * b[i];
            rhs[i + 1] -= f * rhs[i];
        } else {
            const double f = a[i] / c[i];
            a[i] = c[i];
            const double t = a[i + 1];
            a[i + 1] = b[i] - f * t;
            if (i + 2 < n) {
                u2[i] = b[i + 1];
                b[i + 1] = -f * b[i + 1];
            }
            b[i] = t;
            const double r0 = rhs[i];
            rhs[i] = rhs[i + 1];
            rhs[i + 1] = r0 - f * rhs[i + 1];
        }
    }
    if (a[n - 1] == 0.0) a[n - 1] = tiny;
    rhs[n - 1] /= a[n - 1];
    if (n >= 2) rhs[n - 2] = (rhs[n - 2] - b[n - 2] * rhs[n - 1]) / a[n - 2];
    for (int i = n - 3; i >= 0; --i) rhs[i] = (rhs[i] - b[i] * rhs[i + 1] - u2[i] * rhs[i + 2]) / a[i];
}

void sorted_desc(int n, const double* D, std::vector<int>& order) {
    order.resize(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return D[x] > D[y]; });
}

}  // namespace

size_t bidiag_work_doubles(int d) { return (size_t)8 * (d + 2); }

namespace {

// Number of eigenvalues below x[i] of the tridiagonal with diagonal D and squared
// off-diagonal E2, for the m shifts at once: the m pivot recurrences are advanced
// together, so their divisions overlap instead of forming one long chain.
void sturm_counts(const double* D, const double* E2, int n, const double* x, int m, double pivmin, double* dd,
                  int* cnt) {
    for (int i = 0; i < m; ++i) {
        double v = D[0] - x[i];
        if (std::fabs(v) < pivmin) v = -pivmin;
        dd[i] = v;
        cnt[i] = v < 0.0 ? 1 : 0;
    }
    for (int t = 1; t < n; ++t) {
        const double dt = D[t], et = E2[t - 1];
        for (int i = 0; i < m; ++i) {
            double v = dt - x[i] - et / dd[i];
            if (std::fabs(v) < pivmin) v = -pivmin;
            dd[i] = v;
            cnt[i] += v < 0.0 ? 1 : 0;
        }
    }
}

// Squared last component of the unit eigenvector of the tridiagonal at its
// eigenvalue lam, from the twisted factorization of T - lam I (Dhillon and
// Parlett): pivots from the bottom (dm) and from the top (dp), the twist index r
// where |dp_r + dm_r - (D_r - lam)| is least, z_r = 1, and z spread both ways by
// products of pivot ratios.  The tiny last components of converged Ritz vectors
// keep their relative accuracy this way.
double twisted_last2(const double* D, const double* E2, int n, double lam, double pivmin, double* dm, double* dp) {
    if (n == 1) return 1.0;
    auto guard = [pivmin](double x) { return std::fabs(x) < pivmin ? -pivmin : x; };
    dm[n - 1] = D[n - 1] - lam;
    for (int c = n - 2; c >= 0; --c) dm[c] = D[c] - lam - E2[c] / guard(dm[c + 1]);
    double best = 0.0;
    int r = 0;
    for (int c = 0; c < n; ++c) {
        dp[c] = c == 0 ? D[0] - lam : D[c] - lam - E2[c - 1] / guard(dp[c - 1]);
        const double g = std::fabs(dp[c] + dm[c] - (D[c] - lam));
        if (c == 0 || g < best) {
            best = g;
            r = c;
        }
    }
    double z = 1.0, zz = 1.0;
    for (int c = r - 1; c >= 0; --c) {
        z = -(std::sqrt(E2[c]) / guard(dp[c])) * z;
        zz += z * z;
    }
    z = 1.0;
    for (int c = r + 1; c < n; ++c) {
        z = -(std::sqrt(E2[c - 1]) / guard(dm[c])) * z;
        zz += z * z;
    }
    const double zl = r == n - 1 ? 1.0 : z;
    return zl * zl / zz;
}

// The kk largest eigenvalues (descending, into lam) of the tridiagonal with diagonal D
// and off-diagonal E (E[c] couples c and c+1) by bisection on Sturm counts, all kk
// advanced together.  E is replaced by its squares; returns the pivot floor.
double top_eigs_bisect(const double* D, double* E, int n, int kk, double* lam) {
    double gmin = 0.0, gmax = 0.0, e2max = 0.0;
    for (int c = 0; c < n; ++c) {
        const double el = c > 0 ? std::fabs(E[c - 1]) : 0.0, er = c + 1 < n ? std::fabs(E[c]) : 0.0;
        gmin = c == 0 ? D[c] - el - er : std::min(gmin, D[c] - el - er);
        gmax = c == 0 ? D[c] + el + er : std::max(gmax, D[c] + el + er);
    }
    for (int c = 0; c + 1 < n; ++c) {
        E[c] = E[c] * E[c];
        e2max = std::max(e2max, E[c]);
    }
    const double pivmin = 2.2250738585072014e-308 * std::max(1.0, e2max);
    std::vector<double> lo(kk, gmin), hi(kk, gmax), x(kk), dd(kk);
    std::vector<int> cnt(kk);
    const double tolabs = 2.0 * kEps * std::max(std::fabs(gmin), std::fabs(gmax)) + pivmin;
    int rounds = 1;
    for (double w = gmax - gmin; w > tolabs && rounds < 200; w *= 0.5) ++rounds;
    for (int it = 0; it < rounds; ++it) {
        for (int i = 0; i < kk; ++i) x[i] = 0.5 * (lo[i] + hi[i]);
        sturm_counts(D, E, n, x.data(), kk, pivmin, dd.data(), cnt.data());
        for (int i = 0; i < kk; ++i) {
            // the i-th largest eigenvalue is the (n-1-i)-th smallest
            if (cnt[i] <= n - 1 - i)
                lo[i] = x[i];
            else
                hi[i] = x[i];
        }
    }
    for (int i = 0; i < kk; ++i) lam[i] = 0.5 * (lo[i] + hi[i]);
    return pivmin;
}

}  // namespace

void bidiag_ritz_values(const double* alpha, const double* beta, int d, int k, double* omega,
                        double* resid, double* work) {
    if (d >= kBisectMinSteps) {
        // The k largest eigenvalues by bisection on Sturm counts (all k together), their
        // last eigenvector components by twisted factorizations: O(k d) per halving
        // instead of the O(d^2) serial rotations of the full QL iteration.
        double* D = work;
        double* E2 = work + (d + 2);
        double* dm = work + 2 * (d + 2);
        double* dp = work + 3 * (d + 2);
        form_tridiagonal(alpha, beta, d, D, E2);
        const int kk = std::min(k, d);
        std::vector<double> lams(kk);
        const double pivmin = top_eigs_bisect(D, E2, d, kk, lams.data());
        for (int i = 0; i < k; ++i) {
            if (i >= d) {
                omega[i] = 0.0;
                resid[i] = 0.0;
                continue;
            }
            const double lam = lams[i];
            const double w = std::sqrt(std::max(lam, 0.0));
            omega[i] = w;
            const double zl = std::sqrt(twisted_last2(D, E2, d, lam, pivmin, dm, dp));
            resid[i] = w > 0.0 ? alpha[d + 1] * beta[d + 1] * zl / w : 0.0;
        }
        return;
    }
    double* D = work;
    double* E = work + (d + 2);
    double* zl = work + 2 * (d + 2);
    form_tridiagonal(alpha, beta, d, D, E);
    for (int c = 0; c < d; ++c) zl[c] = (c == d - 1) ? 1.0 : 0.0;
    tridiag_ql(d, D, E, zl);
    std::vector<int> order;
    sorted_desc(d, D, order);
    for (int i = 0; i < k; ++i) {
        if (i >= d) {
            omega[i] = 0.0;
            resid[i] = 0.0;
            continue;
        }
        const int o = order[i];
        const double w = std::sqrt(std::max(D[o], 0.0));
        omega[i] = w;
        // alpha_{d+1} |p_i[d]|,  p_i[d] = beta_{d+1} q_i[d-1] / omega_i
        resid[i] = w > 0.0 ? alpha[d + 1] * beta[d + 1] * std::fabs(zl[o]) / w : 0.0;
    }
}

void bidiag_ritz_vectors(const double* alpha, const double* beta, int d, int k, double* omega,
                         double* P, double* Q, double* work) {
    double* D = work;
    double* E = work + (d + 2);
    double* D0 = work + 2 * (d + 2);
    double* E0 = work + 3 * (d + 2);
    double* a = work + 4 * (d + 2);
    double* b = work + 5 * (d + 2);
    double* c = work + 6 * (d + 2);
    double* u2 = work + 7 * (d + 2);
    form_tridiagonal(alpha, beta, d, D0, E0);
    std::memcpy(D, D0, sizeof(double) * d);
    std::memcpy(E, E0, sizeof(double) * d);
    std::vector<int> order;
    if (d >= kBisectMinSteps) {
        // only the k largest eigenvalues are needed: bisection, stored in D[0..k) descending
        const int kq = std::min(k, d);
        std::vector<double> lams(kq);
        top_eigs_bisect(D0, E, d, kq, lams.data());
        for (int i = 0; i < kq; ++i) D[i] = lams[i];
        order.resize(kq);
        for (int i = 0; i < kq; ++i) order[i] = i;
    } else {
        tridiag_ql(d, D, E, nullptr);
        sorted_desc(d, D, order);
    }
    double tnorm = 0.0;
    for (int i = 0; i < d; ++i) tnorm = std::max(tnorm, std::fabs(D0[i]) + 2.0 * std::fabs(i + 1 < d ? E0[i] : 0.0));
    std::vector<double> q((size_t)k * d, 0.0), x(d);
    const int kk = std::min(k, d);
    for (int i = 0; i < kk; ++i) {
        const double lam = D[order[i]];
        // deterministic, generic start vector
        for (int t = 0; t < d; ++t) x[t] = 1.0 + 0.5 * std::sin(0.7 * (t + 1) + 1.3 * (i + 1));
        for (int it = 0; it < 4; ++it) {
            shifted_solve(d, D0, E0, lam, tnorm, x.data(), a, b, c, u2);
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 0; j < i; ++j) {
                    const double* qj = &q[(size_t)j * d];
                    double h = 0.0;
                    for (int t = 0; t < d; ++t) h += qj[t] * x[t];
                    for (int t = 0; t < d; ++t) x[t] -= h * qj[t];
                }
            double nrm = 0.0;
            for (int t = 0; t < d; ++t) nrm += x[t] * x[t];
            nrm = std::sqrt(nrm);
            if (nrm == 0.0) {
                for (int t = 0; t < d; ++t) x[t] = (t == i) ? 1.0 : 0.0;
                nrm = 1.0;
            }
            for (int t = 0; t < d; ++t) x[t] /= nrm;
        }
        std::memcpy(&q[(size_t)i * d], x.data(), sizeof(double) * d);
    }
    double bmax = 0.0;
    for (int r = 0; r < d; ++r) bmax = std::max({bmax, std::fabs(alpha[r + 1]), std::fabs(beta[r + 2])});
    const int n1 = d + 1;
    std::vector<double> pc((size_t)k * n1, 0.0), x1(n1);
    // Gram-Schmidt of x against the left vectors 0..i-1 already chosen (two passes)
    auto orth_prev = [&](int i, double* v) {
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < i; ++j) {
                const double* pj = &pc[(size_t)j * n1];
                double h = 0.0;
                for (int r = 0; r < n1; ++r) h += pj[r] * v[r];
                for (int r = 0; r < n1; ++r) v[r] -= h * pj[r];
            }
        double nrm = 0.0;
        for (int r = 0; r < n1; ++r) nrm += v[r] * v[r];
        return std::sqrt(nrm);
    };
    for (int i = 0; i < k; ++i) {
        omega[i] = i < kk ? std::sqrt(std::max(D[order[i]], 0.0)) : 0.0;
        // Q[t][i] (row-major d x k)
        for (int t = 0; t < d; ++t) Q[(size_t)t * k + i] = i < kk ? q[(size_t)i * d + t] : 0.0;
        // p = B q / omega, normalized and kept orthogonal to the earlier left vectors
        double* p = &pc[(size_t)i * n1];
        if (i < kk) {
            const double* qi = &q[(size_t)i * d];
            for (int r = 0; r <= d; ++r) {
                double v = 0.0;
                if (r < d) v += alpha[r + 1] * qi[r];
                if (r >= 1) v += beta[r + 1] * qi[r - 1];
                p[r] = v;
            }
        }
        double nrm = orth_prev(i, p);
        if (!(nrm > 1e-12 * bmax)) {
            // omega_i = 0 (a series of rank below k): B q vanishes and any unit vector
            // orthogonal to the other left vectors completes the SVD of B
            for (int c = d; c >= 0; --c) {
                std::fill(x1.begin(), x1.end(), 0.0);
                x1[c] = 1.0;
                nrm = orth_prev(i, x1.data());
                if (nrm >= 0.5) {
                    std::copy(x1.begin(), x1.end(), p);
                    break;
                }
            }
        }
        for (int r = 0; r <= d; ++r) {
            p[r] = nrm > 0.0 ? p[r] / nrm : 0.0;
            P[(size_t)r * k + i] = p[r];
        }
    }
}

// Householder vector of x[0..n) (stride sx): on return v[0..n) with v[0] = 1
// and tau such that (I - tau v v^T) x = beta e_0; returns beta.
static double householder(int n, const double* x, long long sx, double* v, double& tau) {
    double s2 = 0.0;
    for (int i = 1; i < n; ++i) s2 += x[(long long)i * sx] * x[(long long)i * sx];
    const double x0 = x[0];
    v[0] = 1.0;
    if (s2 == 0.0) {
        tau = 0.0;
        for (int i = 1; i < n; ++i) v[i] = 0.0;
        return x0;
    }
    const double nrm = std::sqrt(x0 * x0 + s2);
    const double beta = x0 <= 0.0 ? nrm : -nrm;
    const double v0 = x0 - beta;
    for (int i = 1; i < n; ++i) v[i] = x[(long long)i * sx] / v0;
    tau = (beta - x0) / beta;
    return beta;
}

void dense_ritz(const double* A, int nr, int nc, int k, double* omega, double* P, double* Q) {
    // W = A; Golub-Kahan reduction W = Hl [Bu; 0] Hr^T, Bu upper bidiagonal (nc x nc)
    std::vector<double> W(A, A + (size_t)nr * nc);
    std::vector<double> vl((size_t)nc * nr, 0.0), tl(nc, 0.0), vr((size_t)nc * nc, 0.0), tr(nc, 0.0);
    std::vector<double> dg(nc, 0.0), sup(nc, 0.0), tmp(std::max(nr, nc));
    for (int j = 0; j < nc; ++j) {
        double* v = &vl[(size_t)j * nr];
        dg[j] = householder(nr - j, &W[(size_t)j * nc + j], nc, v, tl[j]);
        if (tl[j] != 0.0)
            for (int c = j; c < nc; ++c) {
                double s = 0.0;
                for (int i = j; i < nr; ++i) s += v[i - j] * W[(size_t)i * nc + c];
                s *= tl[j];
                for (int i = j; i < nr; ++i) W[(size_t)i * nc + c] -= s * v[i - j];
            }
        if (j + 1 < nc) {
            double* w = &vr[(size_t)j * nc];
            sup[j] = householder(nc - j - 1, &W[(size_t)j * nc + j + 1], 1, w, tr[j]);
            if (tr[j] != 0.0)
                for (int r = j; r < nr; ++r) {
                    double* row = &W[(size_t)r * nc + j + 1];
                    double s = 0.0;
                    for (int c = 0; c < nc - j - 1; ++c) s += row[c] * w[c];
                    s *= tr[j];
                    for (int c = 0; c < nc - j - 1; ++c) row[c] -= s * w[c];
                }
        }
    }
    // Bu^T is lower bidiagonal: alpha[1..nc] = diagonal, beta[2..nc] = superdiagonal of Bu,
    // beta[nc+1] = 0 (an (nc+1) x nc matrix with a zero last row).
    std::vector<double> al(nc + 3, 0.0), be(nc + 3, 0.0);
    for (int j = 0; j < nc; ++j) al[j + 1] = dg[j];
    for (int j = 0; j + 1 < nc; ++j) be[j + 2] = sup[j];
    const int kk = std::min(k, nc);
    std::vector<double> Pb((size_t)(nc + 1) * kk), Qb((size_t)nc * kk), work(bidiag_work_doubles(nc) + 16);
    bidiag_ritz_vectors(al.data(), be.data(), nc, kk, omega, Pb.data(), Qb.data(), work.data());
    // Bu = Qb diag(omega) Pb[0..nc)^T, so the left vectors of A are Hl [Qb; 0] and the right
    // ones Hr Pb[0..nc); the reflectors are applied last-first to those small blocks.
    std::vector<double> Lft((size_t)nr * kk, 0.0), Rgt((size_t)nc * kk, 0.0);
    for (int i = 0; i < nc; ++i)
        for (int c = 0; c < kk; ++c) {
            Lft[(size_t)i * kk + c] = Qb[(size_t)i * kk + c];
            Rgt[(size_t)i * kk + c] = Pb[(size_t)i * kk + c];
        }
    for (int j = nc - 1; j >= 0; --j) {
        if (tl[j] != 0.0) {
            const double* v = &vl[(size_t)j * nr];
            for (int c = 0; c < kk; ++c) {
                double s = 0.0;
                for (int i = j; i < nr; ++i) s += v[i - j] * Lft[(size_t)i * kk + c];
                s *= tl[j];
                for (int i = j; i < nr; ++i) Lft[(size_t)i * kk + c] -= s * v[i - j];
            }
        }
        if (j + 1 < nc && tr[j] != 0.0) {
            const double* w = &vr[(size_t)j * nc];
            for (int c = 0; c < kk; ++c) {
                double s = 0.0;
                for (int i = j + 1; i < nc; ++i) s += w[i - j - 1] * Rgt[(size_t)i * kk + c];
                s *= tr[j];
                for (int i = j + 1; i < nc; ++i) Rgt[(size_t)i * kk + c] -= s * w[i - j - 1];
            }
        }
    }
    for (int i = 0; i < k; ++i) {
        if (i >= kk) omega[i] = 0.0;
        for (int r = 0; r < nr; ++r) P[(size_t)r * k + i] = i < kk ? Lft[(size_t)r * kk + i] : 0.0;
        for (int r = 0; r < nc; ++r) Q[(size_t)r * k + i] = i < kk ? Rgt[(size_t)r * kk + i] : 0.0;
    }
}

}  // namespace ssa
