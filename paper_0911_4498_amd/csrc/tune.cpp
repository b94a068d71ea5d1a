// tune.cpp -- measured choice of the FFT schedule of the single-series
// products (ssa_tune_fft, ssa_tune_workspace).
//
// Every Lanczos step makes one product X v and one X^T u (Algorithms 2 and 3),
// each a packed-real FFT of M' = M/2 complex points in three passes (columns
// of M1 points, rows of M2 points with the spectral operator, columns again).
// Any M >= N gives the exact correlation (Sec. 4.2), so the transform length
// is free above ceil(N/2) as well as its split and the column blocking.  The
// tuner times the candidates through the public plan API on the caller's
// stream and workspace and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ssa.h"

namespace {

constexpr int kMaxFactor = 4096;  // longest single-workgroup row or column
constexpr int kTuneLengths = 8;   // transform lengths tried, smallest first
constexpr int kTuneSplits = 6;    // splits per length, most balanced first
constexpr double kTuneSpan = 1.25;  // lengths up to 1.25 ceil(N/2)

struct Cand {
    long long mp;
    int m1, cb;
};

bool smooth7(long long n) {
    for (long long p : {2LL, 3LL, 5LL, 7LL})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Schedule candidates for a series of length N: the automatic choice first
// (mp = m1 = cb = 0), then lengths x splits x column blocks.
std::vector<Cand> candidates(long long N) {
    std::vector<Cand> c;
    c.push_back({0, 0, 0});
    const long long m0 = (N + 1) / 2;
    int lengths = 0;
    for (long long mp = m0; mp <= (long long)std::ceil(kTuneSpan * (double)m0) && lengths < kTuneLengths; ++mp) {
        if (!smooth7(mp)) continue;
        std::vector<int> splits;
        for (long long a = 16; a <= kMaxFactor && a <= mp / 16; ++a)
            if (mp % a == 0 && mp / a <= kMaxFactor) splits.push_back((int)a);
        if (splits.empty()) continue;
        ++lengths;
        std::stable_sort(splits.begin(), splits.end(), [mp](int a, int b) {
            return std::fabs(std::log((double)a * a / (double)mp)) < std::fabs(std::log((double)b * b / (double)mp));
        });
        if ((int)splits.size() > kTuneSplits) splits.resize(kTuneSplits);
        for (int m1 : splits) {
            const long long m2 = mp / m1;
            for (int cb : {1, 2, 4, 8})
                if ((long long)cb * m1 <= 8192 && cb <= m2) c.push_back({mp, m1, cb});
        }
    }
    return c;
}

ssa_opts cand_opts(const Cand& c) {
    ssa_opts o{};
    o.d_max = 2;
    o.fft_mp = c.mp;
    o.fft_m1 = c.m1;
    o.fft_cb = c.cb;
    return o;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Bytes of the product vectors behind the plan region: x (K), y (L), x' (L), y' (K).
size_t vec_bytes(long long L, long long K) { return 2 * align256(sizeof(float) * (size_t)(L + K)); }

}  // namespace

extern "C" {

int ssa_tune_workspace(long long N, long long L, size_t* bytes) {
    if (!bytes || N < 3 || L < 2 || L >= N) return SSA_EINVAL;
    size_t most = 0;
    for (const Cand& c : candidates(N)) {
        const ssa_opts o = cand_opts(c);
        size_t ws = 0;
        ssa_plan p = nullptr;
        if (ssa_embed_plan(N, L, 1, &o, &ws, &p) != SSA_OK) continue;
        ssa_plan_destroy(p);
        most = std::max(most, ws);
    }
    if (most == 0) return SSA_EINVAL;
    *bytes = align256(most) + vec_bytes(L, N - L + 1);
    return SSA_OK;
}

int ssa_tune_fft(long long N, long long L, const double* series_dev, void* workspace_dev, size_t bytes,
                 void* hip_stream, int reps, ssa_opts* best, double* us_best, int max_rows, long long* rows,
                 double* us, int* nrows) {
    if (!series_dev || !workspace_dev || !best || reps < 1 || max_rows < 0 || (max_rows > 0 && (!rows || !us)))
        return SSA_EINVAL;
    size_t need = 0;
    int rc = ssa_tune_workspace(N, L, &need);
    if (rc != SSA_OK) return rc;
    if (bytes < need || ((uintptr_t)workspace_dev & 255) != 0) return SSA_ENOMEM;
    const long long K = N - L + 1;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char* base = static_cast<char*>(workspace_dev);
    const size_t plan_bytes = need - vec_bytes(L, K);
    float* x = reinterpret_cast<float*>(base + plan_bytes);  // K entries, then y (L)
    float* y = x + K;
    float* xt = reinterpret_cast<float*>(base + plan_bytes + align256(sizeof(float) * (size_t)(L + K)));
    float* yt = xt + L;  // L entries of x', then K of y'
    if (hipMemsetAsync(base + plan_bytes, 0, vec_bytes(L, K), s) != hipSuccess) return SSA_EDEVICE;
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) return SSA_EDEVICE;
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return SSA_EDEVICE;
    }
    double best_us = INFINITY;
    Cand best_c{0, 0, 0};
    int timed = 0;
    rc = SSA_OK;
    for (const Cand& c : candidates(N)) {
        const ssa_opts o = cand_opts(c);
        size_t ws = 0;
        ssa_plan p = nullptr;
        if (ssa_embed_plan(N, L, 1, &o, &ws, &p) != SSA_OK) continue;
        ssa_plan_desc d{};
        double t = INFINITY;
        int prc = ssa_plan_describe(p, &d);
        if (prc == SSA_OK) prc = ssa_plan_bind(p, workspace_dev, plan_bytes, hip_stream);
        if (prc == SSA_OK) prc = ssa_embed(p, series_dev);
        for (int w = 0; w < 2 && prc == SSA_OK; ++w) {  // warm-up
            prc = ssa_matvec(p, 0, x, y);
            if (prc == SSA_OK) prc = ssa_matvec(p, 1, xt, yt);
        }
        for (int run = 0; run < 3 && prc == SSA_OK; ++run) {
            if (hipEventRecord(ev[0], s) != hipSuccess) prc = SSA_EDEVICE;
            for (int i = 0; i < reps && prc == SSA_OK; ++i) {
                prc = ssa_matvec(p, 0, x, y);
                if (prc == SSA_OK) prc = ssa_matvec(p, 1, xt, yt);
            }
            if (prc == SSA_OK && hipEventRecord(ev[1], s) != hipSuccess) prc = SSA_EDEVICE;
            float ms = 0.0f;
            if (prc == SSA_OK && (hipEventSynchronize(ev[1]) != hipSuccess ||
                                  hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
                prc = SSA_EDEVICE;
            if (prc == SSA_OK) t = std::min(t, 1000.0 * (double)ms / (double)reps);
        }
        ssa_plan_destroy(p);
        if (prc != SSA_OK) {
            rc = prc;
            break;
        }
        if (timed < max_rows) {
            rows[3 * timed] = d.M / 2;
            rows[3 * timed + 1] = d.M1;
            rows[3 * timed + 2] = d.cb;
            us[timed] = t;
        }
        ++timed;
        if (t < best_us) {
            best_us = t;
            best_c = {d.M / 2, (int)d.M1, d.cb};
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc != SSA_OK) return rc;
    if (timed == 0) return SSA_EINVAL;
    best->fft_mp = best_c.mp;
    best->fft_m1 = best_c.m1;
    best->fft_cb = best_c.cb;
    if (us_best) *us_best = best_us;
    if (nrows) *nrows = timed;
    return SSA_OK;
}

}  // extern "C"
