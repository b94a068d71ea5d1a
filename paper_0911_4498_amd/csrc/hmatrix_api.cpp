// hmatrix_api.cpp -- workloads built on the many-series engine:
//  * ssa_hmatrix: structural-change detection by the H-matrix of heterogeneity
//    indices (eq. g); the SSAs of all base windows run as one batch, the
//    indices come from the kernels of hmatrix.hip;
//  * ssa_realizations: statistics of rank-d reconstructions over repeated
//    realizations of a series (realizations.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "ssa.h"
#include "ssa_batch.h"
#include "ssa_hmatrix.h"

using namespace ssa;

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct HmLayout {
    long long MB, MT, P, K2, KB;
    int k;
    size_t o_win, o_U, o_sig, o_V, o_I, o_sq, o_c2, o_batch, batch_bytes, total;
};

// Validates the arguments and lays out the workspace; false on invalid input.
bool hm_layout(long long N, long long B, long long T, long long L, const int* I, int nI, HmLayout& h,
               ssa_batch* engine) {
    if (!I || nI < 1 || nI > batch::kMaxK || N < 4 || B > N || T > N || L <= 1 || L >= B - 1 || L > T) return false;
    if (B > 2LL * batch::kMaxMp) return false;
    int k = 0;
    for (int q = 0; q < nI; ++q) {
        if (I[q] < 1 || I[q] > batch::kMaxK) return false;
        k = std::max(k, I[q]);
    }
    h.KB = B - L + 1;
    if (k > std::min(L, h.KB)) return false;
    // the correlation kernel holds nI eigenvectors and a tile of the series in LDS
    if (sizeof(float) * ((size_t)nI * L + 256 + L) > 160 * 1024) return false;
    h.k = k;
    h.MB = N - B + 1;
    h.MT = N - T + 1;
    h.P = N - L + 1;
    h.K2 = T - L + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    h.o_win = take(sizeof(double) * (size_t)(h.MB * B));
    h.o_U = take(sizeof(float) * (size_t)(h.MB * L * k));
    h.o_sig = take(sizeof(double) * (size_t)(h.MB * k));
    h.o_V = take(sizeof(float) * (size_t)(h.MB * h.KB * k));
    h.o_I = take(sizeof(int) * (size_t)nI);
    h.o_sq = take(sizeof(double) * (size_t)h.P);
    h.o_c2 = take(sizeof(double) * (size_t)(h.MB * h.P));
    ssa_batch b = nullptr;
    size_t bound = 0;
    if (ssa_batch_plan(B, k, (int)h.MB, nullptr, &bound, &b) != SSA_OK) return false;
    std::vector<long long> offs(h.MB + 1);
    for (long long i = 0; i <= h.MB; ++i) offs[i] = i * B;
    std::vector<int> Ls(h.MB, (int)L), ks(h.MB, k);
    size_t need = 0;
    if (ssa_batch_workspace(b, (int)h.MB, offs.data(), Ls.data(), ks.data(), &need) != SSA_OK) {
        ssa_batch_destroy(b);
        return false;
    }
    h.o_batch = take(need);
    h.batch_bytes = need;
    h.total = o;
    if (engine)
        *engine = b;
    else
        ssa_batch_destroy(b);
    return true;
}

}  // namespace

extern "C" {

int ssa_hmatrix_workspace(long long N, long long B, long long T, long long L, const int* I, int nI, size_t* bytes) {
    if (!bytes) return SSA_EINVAL;
    HmLayout h;
    if (!hm_layout(N, B, T, L, I, nI, h, nullptr)) return SSA_EINVAL;
    *bytes = h.total;
    return SSA_OK;
}

int ssa_hmatrix(const double* series_dev, long long N, long long B, long long T, long long L, const int* I, int nI,
                void* workspace_dev, size_t bytes, void* hip_stream, double* G_dev) {
    if (!series_dev || !workspace_dev || !G_dev) return SSA_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256) return SSA_EINVAL;
    HmLayout h;
    ssa_batch eng = nullptr;
    if (!hm_layout(N, B, T, L, I, nI, h, &eng)) return SSA_EINVAL;
    if (bytes < h.total) {
        ssa_batch_destroy(eng);
        return SSA_ENOMEM;
    }
    char* ws = static_cast<char*>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* win = reinterpret_cast<double*>(ws + h.o_win);
    float* U = reinterpret_cast<float*>(ws + h.o_U);
    int* dI = reinterpret_cast<int*>(ws + h.o_I);
    double* sq = reinterpret_cast<double*>(ws + h.o_sq);
    double* c2 = reinterpret_cast<double*>(ws + h.o_c2);
    int rc = SSA_OK;
    std::vector<long long> offs(h.MB + 1);
    for (long long i = 0; i <= h.MB; ++i) offs[i] = i * B;
    std::vector<int> Ls(h.MB, (int)L), ks(h.MB, h.k);
    std::vector<unsigned long long> keys(h.MB);
    for (long long i = 0; i < h.MB; ++i) keys[i] = (unsigned long long)i;
    do {
        if (hipMemcpyAsync(dI, I, sizeof(int) * (size_t)nI, hipMemcpyHostToDevice, s) != hipSuccess ||
            launch_hm_windows(series_dev, B, h.MB, win, s) != hipSuccess) {
            rc = SSA_EDEVICE;
            break;
        }
        // every base window's leading k eigenvectors (the batched path); U is L x k per window
        rc = ssa_batch_bind(eng, ws + h.o_batch, h.batch_bytes, hip_stream);
        if (rc != SSA_OK) break;
        rc = ssa_batch_solve(eng, (int)h.MB, win, offs.data(), Ls.data(), ks.data(), keys.data(),
                             reinterpret_cast<double*>(ws + h.o_sig), U, reinterpret_cast<float*>(ws + h.o_V),
                             nullptr, nullptr);
        if (rc != SSA_OK) break;
        if (launch_hm_corr(series_dev, N, L, U, h.k, dI, nI, h.MB, c2, s) != hipSuccess ||
            launch_hm_energy(series_dev, N, L, sq, s) != hipSuccess ||
            launch_hm_rows(c2, sq, h.P, h.MB, h.MT, h.K2, G_dev, s) != hipSuccess) {
            rc = SSA_EDEVICE;
            break;
        }
        // the call returns with G complete (the host arrays above are then free to go)
        if (hipStreamSynchronize(s) != hipSuccess) rc = SSA_EDEVICE;
    } while (false);
    ssa_batch_destroy(eng);
    return rc;
}

}  // extern "C"

namespace {

struct RsLayout {
    long long KL;
    size_t o_sig, o_U, o_V, o_rec, o_batch, batch_bytes, total;
};

bool rs_layout(long long R, long long N, long long L, int d, RsLayout& h, ssa_batch* engine) {
    if (R < 1 || R > (1LL << 20) || N < 3 || N > 2LL * batch::kMaxMp || L <= 1 || L >= N || d < 1 ||
        d > batch::kMaxK)
        return false;
    const long long K = N - L + 1;
    if (d > std::min(L, K)) return false;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    h.o_sig = take(sizeof(double) * (size_t)(R * d));
    h.o_U = take(sizeof(float) * (size_t)(R * L * d));
    h.o_V = take(sizeof(float) * (size_t)(R * K * d));
    h.o_rec = take(sizeof(float) * (size_t)(R * N * d));
    ssa_batch b = nullptr;
    size_t bound = 0;
    if (ssa_batch_plan(N, d, (int)R, nullptr, &bound, &b) != SSA_OK) return false;
    std::vector<long long> offs(R + 1);
    for (long long r = 0; r <= R; ++r) offs[r] = r * N;
    std::vector<int> Ls(R, (int)L), ks(R, d);
    size_t need = 0;
    if (ssa_batch_workspace(b, (int)R, offs.data(), Ls.data(), ks.data(), &need) != SSA_OK) {
        ssa_batch_destroy(b);
        return false;
    }
    h.o_batch = take(need);
    h.batch_bytes = need;
    h.total = o;
    if (engine)
        *engine = b;
    else
        ssa_batch_destroy(b);
    return true;
}

}  // namespace

extern "C" {

int ssa_realizations_workspace(long long R, long long N, long long L, int d, size_t* bytes) {
    if (!bytes) return SSA_EINVAL;
    RsLayout h;
    if (!rs_layout(R, N, L, d, h, nullptr)) return SSA_EINVAL;
    *bytes = h.total;
    return SSA_OK;
}

int ssa_realizations(const double* series_dev, long long R, long long N, long long L, int d, const double* truth_dev,
                     void* workspace_dev, size_t bytes, void* hip_stream, double* mean_dev, double* var_dev,
                     double* mse_dev) {
    if (!series_dev || !workspace_dev || !mean_dev || !var_dev || (mse_dev && !truth_dev)) return SSA_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256) return SSA_EINVAL;
    RsLayout h;
    ssa_batch eng = nullptr;
    if (!rs_layout(R, N, L, d, h, &eng)) return SSA_EINVAL;
    if (bytes < h.total) {
        ssa_batch_destroy(eng);
        return SSA_ENOMEM;
    }
    char* ws = static_cast<char*>(workspace_dev);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float* rec = reinterpret_cast<float*>(ws + h.o_rec);
    std::vector<long long> offs(R + 1);
    for (long long r = 0; r <= R; ++r) offs[r] = r * N;
    std::vector<int> Ls(R, (int)L), ks(R, d);
    std::vector<unsigned long long> keys(R);
    for (long long r = 0; r < R; ++r) keys[r] = (unsigned long long)r;
    int rc = ssa_batch_bind(eng, ws + h.o_batch, h.batch_bytes, hip_stream);
    if (rc == SSA_OK)
        rc = ssa_batch_solve(eng, (int)R, series_dev, offs.data(), Ls.data(), ks.data(), keys.data(),
                             reinterpret_cast<double*>(ws + h.o_sig), reinterpret_cast<float*>(ws + h.o_U),
                             reinterpret_cast<float*>(ws + h.o_V), rec, nullptr);
    if (rc == SSA_OK &&
        (launch_realization_stats(rec, R, d, N, truth_dev, mean_dev, var_dev, mse_dev, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        rc = SSA_EDEVICE;
    ssa_batch_destroy(eng);
    return rc;
}

}  // extern "C"
