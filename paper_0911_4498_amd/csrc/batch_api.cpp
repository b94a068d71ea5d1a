// batch_api.cpp -- C ABI of the many-series engine (ssa_batch_*): builds the
// per-series table and region layout, validates, and drives the lockstep
// launches of batch.hip (one launch per Lanczos half-step for the whole batch,
// a stopping-test launch at check points, then Ritz triples and Hankelization).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <set>
#include <vector>

#include "ssa.h"
#include "ssa_batch.h"
#include "ssa_internal.h"

using namespace ssa;

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool smooth7(long long m) {
    for (int p : {2, 3, 5, 7})
        while (m % p == 0) m /= p;
    return m == 1;
}

FftStages plan_radices(int n) {
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

// splitmix64 finalizer: per-series seed from the batch seed and the series key
unsigned long long mix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

}  // namespace

struct ssa_batch_s {
    long long n_max;
    int k_max, d_max, check_every, max_series;
    double tol;
    unsigned long long seed;
    size_t tab_bytes, t_ndone, regions_off, bound_bytes;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int bound = 0;
    BSeries* h_tab = nullptr;     // pinned staging of the series table
    unsigned* h_done = nullptr;   // pinned, double-buffered finished-series counts
    hipEvent_t tab_done = nullptr;
    hipEvent_t chk_ev[2] = {nullptr, nullptr};
    std::vector<BSeries> tab;
    // optional HIP-event timing of the kernel classes in prof_mask
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> prof_events;
    size_t prof_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pairs[SSA_BPROF_NCLASSES];
    long long prof_count[SSA_BPROF_NCLASSES] = {};
};

namespace {

// Fill b->tab for these series; returns the workspace bytes they need, or 0 on invalid input.
size_t build_table(ssa_batch b, int nseries, const long long* offsets, const int* L, const int* k,
                   const unsigned long long* keys) {
    if (nseries < 1 || nseries > b->max_series || !offsets || !L || !k || offsets[0] != 0) return 0;
    b->tab.assign(nseries, BSeries{});
    size_t off = b->regions_off;
    for (int s = 0; s < nseries; ++s) {
        const long long N = offsets[s + 1] - offsets[s];
        if (N < 3 || N > b->n_max) return 0;
        if (L[s] <= 1 || L[s] >= N) return 0;
        const long long K = N - L[s] + 1;
        const long long r = std::min<long long>(L[s], K);
        if (k[s] < 1 || k[s] > b->k_max || k[s] > r) return 0;
        BSeries& t = b->tab[s];
        t.f_off = offsets[s];
        t.N = N;
        t.L = L[s];
        t.k = k[s];
        t.transposed = L[s] > K ? 1 : 0;
        t.Li = std::min<long long>(L[s], K);
        t.Ki = std::max<long long>(L[s], K);
        long long mp = (N + 1) / 2;
        while (!smooth7(mp)) ++mp;
        if (mp > batch::kMaxMp) return 0;
        t.Mp = (int)mp;
        int shift = 0;
        while ((1LL << (2 * shift)) < mp) ++shift;
        t.tw_shift = shift;
        t.st = plan_radices(t.Mp);
        int dmax = b->d_max > 0 ? b->d_max : 8 * k[s] + 32;
        dmax = std::min(dmax, batch::kDmax);
        t.dcap = (int)std::max<long long>(k[s], std::min<long long>(dmax, r));
        t.ldu = (long long)align_up((size_t)t.Li, 64);
        t.ldv = (long long)align_up((size_t)t.Ki, 64);
        const unsigned long long key = keys ? keys[s] : (unsigned long long)s;
        t.seed = mix64(b->seed ^ mix64(key));
        size_t o = 0;
        auto take = [&](size_t bytes) {
            const size_t at = o;
            o = align_up(o + bytes, 256);
            return (long long)at;
        };
        const size_t dc = (size_t)t.dcap;
        t.o_ab = take(sizeof(float4) * (size_t)t.Mp);
        t.o_tw = take(sizeof(float2) * 2 * batch::kTwTab);
        t.o_u = take(sizeof(float) * (dc + 1) * (size_t)t.ldu);
        t.o_v = take(sizeof(float) * (dc + 1) * (size_t)t.ldv);
        t.o_r = take(sizeof(float) * (size_t)t.ldv);  // product / Gram-Schmidt vector (Ki >= Li entries)
        t.o_alpha = take(sizeof(double) * (dc + 3));
        t.o_beta = take(sizeof(double) * (dc + 3));
        t.o_state = take(sizeof(double) * batch::kStDoubles);
        t.o_p = take(sizeof(double) * (dc + 1) * (size_t)t.k);
        t.o_q = take(sizeof(double) * dc * (size_t)t.k);
        t.o_scr = take(std::max(sizeof(double) * (size_t)t.k * 5 * (dc + 2), sizeof(float2) * (size_t)t.Mp));
        t.reg = (long long)off;
        off += o;
    }
    // output offsets, in input order
    long long so = 0, uo = 0, vo = 0, ro = 0;
    for (int s = 0; s < nseries; ++s) {
        BSeries& t = b->tab[s];
        const long long K = t.N - t.L + 1;
        t.s_off = so;
        t.u_off = uo;
        t.v_off = vo;
        t.r_off = ro;
        so += t.k;
        uo += (long long)t.L * t.k;
        vo += K * t.k;
        ro += t.N * t.k;
    }
    return off;
}

hipEvent_t prof_event(ssa_batch b) {
    if (b->prof_used == b->prof_events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        b->prof_events.push_back(e);
    }
    return b->prof_events[b->prof_used++];
}

// Enqueue one launch of class cls, bracketed by events when that class is timed.
template <typename F>
hipError_t timed(ssa_batch b, int cls, F&& launch) {
    hipEvent_t e0 = (b->prof_mask >> cls & 1u) ? prof_event(b) : nullptr;
    if (e0 && hipEventRecord(e0, b->stream) != hipSuccess) return hipErrorUnknown;
    const hipError_t e = launch();
    if (e != hipSuccess) return e;
    b->prof_count[cls] += 1;
    if (e0) {
        hipEvent_t e1 = prof_event(b);
        if (!e1 || hipEventRecord(e1, b->stream) != hipSuccess) return hipErrorUnknown;
        b->prof_pairs[cls].push_back({e0, e1});
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int ssa_batch_plan(long long n_max, int k_max, int max_series, const ssa_opts* opts, size_t* workspace_bytes,
                   ssa_batch* out) {
    if (!out || !workspace_bytes) return SSA_EINVAL;
    *out = nullptr;
    if (n_max < 3 || n_max > 2LL * batch::kMaxMp || k_max < 1 || k_max > batch::kMaxK || max_series < 1)
        return SSA_EINVAL;
    ssa_batch b = new (std::nothrow) ssa_batch_s();
    if (!b) return SSA_EINVAL;
    b->n_max = n_max;
    b->k_max = k_max;
    b->max_series = max_series;
    b->d_max = opts && opts->d_max > 0 ? std::min(opts->d_max, batch::kDmax) : 0;
    b->check_every = opts && opts->check_every > 0 ? opts->check_every : 4;
    b->tol = opts && opts->tol > 0.0 ? opts->tol : 1e-8;
    b->seed = opts && opts->seed ? opts->seed : 1ULL;
    b->tab_bytes = align_up(sizeof(BSeries) * (size_t)max_series, 256);
    b->t_ndone = b->tab_bytes;
    b->regions_off = b->t_ndone + 256;
    // bound: max_series series of length n_max with L = n_max / 2 and k = k_max
    std::vector<long long> offs(max_series + 1);
    std::vector<int> Ls(max_series, (int)(n_max / 2)), ks(max_series, (int)std::min<long long>(k_max, n_max / 2));
    for (int s = 0; s <= max_series; ++s) offs[s] = (long long)s * n_max;
    const size_t need = build_table(b, max_series, offs.data(), Ls.data(), ks.data(), nullptr);
    b->tab.clear();
    if (need == 0) {
        delete b;
        return SSA_EINVAL;
    }
    b->bound_bytes = need;
    *workspace_bytes = need;
    *out = b;
    return SSA_OK;
}

int ssa_batch_workspace(ssa_batch b, int nseries, const long long* offsets, const int* L, const int* k,
                        size_t* bytes) {
    if (!b || !bytes) return SSA_EINVAL;
    const size_t need = build_table(b, nseries, offsets, L, k, nullptr);
    b->tab.clear();
    if (need == 0) return SSA_EINVAL;
    *bytes = need;
    return SSA_OK;
}

int ssa_batch_bind(ssa_batch b, void* workspace_dev, size_t bytes, void* hip_stream) {
    if (!b || !workspace_dev) return SSA_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256) return SSA_EINVAL;
    if (bytes < b->regions_off) return SSA_ENOMEM;
    if (!b->h_tab) {
        if (hipHostMalloc((void**)&b->h_tab, sizeof(BSeries) * (size_t)b->max_series, hipHostMallocDefault) !=
            hipSuccess)
            return SSA_EDEVICE;
        if (hipHostMalloc((void**)&b->h_done, sizeof(unsigned) * 2, hipHostMallocDefault) != hipSuccess)
            return SSA_EDEVICE;
        if (hipEventCreateWithFlags(&b->tab_done, hipEventDisableTiming) != hipSuccess) return SSA_EDEVICE;
        for (hipEvent_t& e : b->chk_ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return SSA_EDEVICE;
    }
    b->ws = static_cast<char*>(workspace_dev);
    b->ws_bytes = bytes;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->bound = 1;
    return SSA_OK;
}

#define SSA_TRY_HIP(x)                             \
    do {                                           \
        if ((x) != hipSuccess) return SSA_EDEVICE; \
    } while (0)

int ssa_batch_solve(ssa_batch b, int nseries, const double* series_dev, const long long* offsets, const int* L,
                    const int* k, const unsigned long long* keys, double* sigma_dev, float* U_dev, float* V_dev,
                    float* recon_dev, int* info_dev) {
    if (!b || !series_dev || !offsets || !L || !k || !sigma_dev || !U_dev || !V_dev) return SSA_EINVAL;
    const size_t need = build_table(b, nseries, offsets, L, k, keys);
    if (need == 0) return SSA_EINVAL;
    if (!b->bound || need > b->ws_bytes) return SSA_ENOMEM;
    hipStream_t st = b->stream;
    // the previous solve's table upload must be done before the staging is reused
    SSA_TRY_HIP(hipEventSynchronize(b->tab_done));
    std::memcpy(b->h_tab, b->tab.data(), sizeof(BSeries) * (size_t)nseries);
    SSA_TRY_HIP(hipMemcpyAsync(b->ws, b->h_tab, sizeof(BSeries) * (size_t)nseries, hipMemcpyHostToDevice, st));
    SSA_TRY_HIP(hipEventRecord(b->tab_done, st));
    SSA_TRY_HIP(launch_fill_zero(reinterpret_cast<double*>(b->ws + b->t_ndone), 1, st));

    BatchArgs a{};
    a.nseries = nseries;
    a.tab = reinterpret_cast<const BSeries*>(b->ws);
    a.series = series_dev;
    a.ws = b->ws;
    a.sigma = sigma_dev;
    a.U = U_dev;
    a.V = V_dev;
    a.recon = recon_dev;
    a.info = info_dev;
    a.ndone = reinterpret_cast<unsigned*>(b->ws + b->t_ndone);
    a.check_every = b->check_every;
    a.tol = b->tol;

    int kmin = b->tab[0].k, maxcap = 0;
    std::set<int> caps;
    for (const BSeries& t : b->tab) {
        kmin = std::min(kmin, t.k);
        maxcap = std::max(maxcap, t.dcap);
        caps.insert(t.dcap);
    }
    SSA_TRY_HIP(timed(b, SSA_BPROF_INIT, [&] { return launch_batch_init(a, st); }));
    // Lanczos steps in lockstep.  The finished-series count of one check is read
    // while the GPU runs the steps enqueued after it, so the host never waits on
    // the GPU; once every series is finished, the steps already enqueued find
    // nothing left to do.
    int pend = -1, cur = 0;
    for (int j = 1; j <= maxcap + 1; ++j) {
        const int jj = j - 1;
        SSA_TRY_HIP(timed(b, SSA_BPROF_CONV, [&] { return launch_batch_conv(a, j, 0, st); }));
        SSA_TRY_HIP(timed(b, SSA_BPROF_CGS, [&] { return launch_batch_cgs(a, j, 0, st); }));
        bool stop = false;
        if (jj >= kmin && (jj % b->check_every == 0 || caps.count(jj))) {
            SSA_TRY_HIP(timed(b, SSA_BPROF_CHECK, [&] { return launch_batch_check(a, j, st); }));
            SSA_TRY_HIP(hipMemcpyAsync(b->h_done + cur, a.ndone, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            SSA_TRY_HIP(hipEventRecord(b->chk_ev[cur], st));
            if (pend >= 0) {
                SSA_TRY_HIP(hipEventSynchronize(b->chk_ev[pend]));
                stop = b->h_done[pend] >= (unsigned)nseries;
            }
            pend = cur;
            cur ^= 1;
        }
        if (stop || jj >= maxcap) break;
        SSA_TRY_HIP(timed(b, SSA_BPROF_CONV, [&] { return launch_batch_conv(a, j, 1, st); }));
        SSA_TRY_HIP(timed(b, SSA_BPROF_CGS, [&] { return launch_batch_cgs(a, j, 1, st); }));
    }
    SSA_TRY_HIP(timed(b, SSA_BPROF_RITZ, [&] { return launch_batch_ritz(a, st); }));
    if (recon_dev) SSA_TRY_HIP(timed(b, SSA_BPROF_HANKEL, [&] { return launch_batch_hankel(a, st); }));
    return SSA_OK;
}

int ssa_batch_profile_enable(ssa_batch b, unsigned class_mask) {
    if (!b) return SSA_EINVAL;
    if (b->bound && hipStreamSynchronize(b->stream) != hipSuccess) return SSA_EDEVICE;
    for (int c = 0; c < SSA_BPROF_NCLASSES; ++c) {
        b->prof_pairs[c].clear();
        b->prof_count[c] = 0;
    }
    b->prof_used = 0;
    b->prof_mask = class_mask;
    return SSA_OK;
}

int ssa_batch_profile_read(ssa_batch b, int cls, long long* launches, double* ms) {
    if (!b || cls < 0 || cls >= SSA_BPROF_NCLASSES) return SSA_EINVAL;
    if (b->bound && hipStreamSynchronize(b->stream) != hipSuccess) return SSA_EDEVICE;
    double total = 0.0;
    for (auto& pr : b->prof_pairs[cls]) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess) return SSA_EDEVICE;
        total += t;
    }
    if (launches) *launches = b->prof_count[cls];
    if (ms) *ms = (b->prof_mask >> cls & 1u) ? total : -1.0;
    return SSA_OK;
}

void ssa_batch_destroy(ssa_batch b) {
    if (!b) return;
    if (b->tab_done) {
        (void)hipEventSynchronize(b->tab_done);
        (void)hipEventDestroy(b->tab_done);
    }
    for (hipEvent_t e : b->chk_ev)
        if (e) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
    for (hipEvent_t e : b->prof_events) (void)hipEventDestroy(e);
    if (b->h_tab) (void)hipHostFree(b->h_tab);
    if (b->h_done) (void)hipHostFree(b->h_done);
    delete b;
}

}  // extern "C"

static_assert(sizeof(BSeries) % 8 == 0, "series table entries must keep 8-byte alignment");
static_assert(2 * batch::kMaxMp <= batch::kEpt * batch::kThreads * 2, "in-LDS FFT needs M' <= EPT * threads");
