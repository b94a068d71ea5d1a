// batch_api.cpp -- C ABI of the many-series engine (ssa_batch_*) and of the
// continuous-batching server built on the same kernels (ssa_server_*).
//
// Both lay out one region per series in the caller's workspace (spectral
// operator, twiddles, Lanczos bases, alpha/beta, stopping-test state) and
// describe it to the kernels of batch.hip in a table of BSeries.  Every
// launch covers a list of series with one workgroup each; each series carries
// its own Lanczos step, so series can start and finish at different launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <set>
#include <thread>
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

// splitmix64 finalizer: per-series seed from the engine seed and the series key
unsigned long long mix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

struct EngineCfg {
    long long n_max;
    int k_max, d_max, check_every;
    double tol;
    unsigned long long seed;
    int onesided;
};

// Geometry and region layout of one series; returns its region bytes (offsets
// relative to the region), or 0 if the series is invalid for this engine.
size_t layout_series(const EngineCfg& c, long long N, long long L, int k, unsigned long long key, BSeries& t) {
    if (N < 3 || N > c.n_max || L <= 1 || L >= N) return 0;
    const long long K = N - L + 1;
    const long long r = std::min(L, K);
    if (k < 1 || k > c.k_max || k > r) return 0;
    t = BSeries{};
    t.N = N;
    t.L = (int)L;
    t.k = k;
    t.transposed = L > K ? 1 : 0;
    t.Li = std::min(L, K);
    t.Ki = std::max(L, K);
    long long mp = (N + 1) / 2;
    while (!smooth7(mp)) ++mp;
    if (mp > batch::kMaxMp) return 0;
    t.Mp = (int)mp;
    int shift = 0;
    while ((1LL << (2 * shift)) < mp) ++shift;
    t.tw_shift = shift;
    t.st = plan_radices(t.Mp);
    int dmax = c.d_max > 0 ? c.d_max : 8 * k + 32;
    dmax = std::min(dmax, batch::kDmax);
    t.dcap = (int)std::max<long long>(k, std::min<long long>(dmax, r));
    t.ldu = (long long)align_up((size_t)t.Li, 64);
    t.ldv = (long long)align_up((size_t)t.Ki, 64);
    t.seed = mix64(c.seed ^ mix64(key));
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
    return o;
}

EngineCfg make_cfg(long long n_max, int k_max, const ssa_opts* opts) {
    EngineCfg c{};
    c.n_max = n_max;
    c.k_max = k_max;
    c.d_max = opts && opts->d_max > 0 ? std::min(opts->d_max, batch::kDmax) : 0;
    c.check_every = opts && opts->check_every > 0 ? opts->check_every : 4;
    c.tol = opts && opts->tol > 0.0 ? opts->tol : 1e-8;
    c.seed = opts && opts->seed ? opts->seed : 1ULL;
    c.onesided = opts && opts->reorth == 1 ? 1 : 0;
    return c;
}

// thick restart is a single-series option; reorth is 0 (full) or 1 (one-sided)
bool cfg_valid(long long n_max, int k_max, const ssa_opts* opts) {
    if (opts && (opts->restart_keep != 0 || (opts->reorth != 0 && opts->reorth != 1))) return false;
    return n_max >= 3 && n_max <= 2LL * batch::kMaxMp && k_max >= 1 && k_max <= batch::kMaxK;
}

#define SSA_TRY_HIP(x)                             \
    do {                                           \
        if ((x) != hipSuccess) return SSA_EDEVICE; \
    } while (0)

}  // namespace

// ===========================================================================
// batch engine: a fixed set of series solved to completion by one call

struct ssa_batch_s {
    EngineCfg cfg;
    int max_series;
    size_t tab_bytes, t_ndone, regions_off;
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
        const size_t bytes = layout_series(b->cfg, N, L[s], k[s], keys ? keys[s] : (unsigned long long)s, b->tab[s]);
        if (bytes == 0) return 0;
        b->tab[s].reg = (long long)off;
        off += bytes;
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
    if (!cfg_valid(n_max, k_max, opts) || max_series < 1) return SSA_EINVAL;
    ssa_batch b = new (std::nothrow) ssa_batch_s();
    if (!b) return SSA_EINVAL;
    b->cfg = make_cfg(n_max, k_max, opts);
    b->max_series = max_series;
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

int ssa_batch_solve(ssa_batch b, int nseries, const double* series_dev, const long long* offsets, const int* L,
                    const int* k, const unsigned long long* keys, double* sigma_dev, float* U_dev, float* V_dev,
                    float* recon_dev, int* info_dev) {
    if (!b || !series_dev || !offsets || !L || !k || !sigma_dev || !U_dev || !V_dev) return SSA_EINVAL;
    const size_t need = build_table(b, nseries, offsets, L, k, keys);
    if (need == 0) return SSA_EINVAL;
    if (!b->bound || need > b->ws_bytes) return SSA_ENOMEM;
    // outputs: one block per series in input order
    long long so = 0, uo = 0, vo = 0, ro = 0;
    for (int s = 0; s < nseries; ++s) {
        BSeries& t = b->tab[s];
        const long long K = t.N - t.L + 1;
        t.f = series_dev + offsets[s];
        t.sigma = sigma_dev + so;
        t.U = U_dev + uo;
        t.V = V_dev + vo;
        t.recon = recon_dev ? recon_dev + ro : nullptr;
        t.info = info_dev ? info_dev + 4LL * s : nullptr;
        so += t.k;
        uo += (long long)t.L * t.k;
        vo += K * t.k;
        ro += t.N * t.k;
    }
    // one workgroup per table entry: the longest series first, so that the short ones fill
    // the tail of every launch (each entry carries its own region and output pointers)
    std::stable_sort(b->tab.begin(), b->tab.end(), [](const BSeries& x, const BSeries& y) { return x.N > y.N; });
    hipStream_t st = b->stream;
    // the previous solve's table upload must be done before the staging is reused
    SSA_TRY_HIP(hipEventSynchronize(b->tab_done));
    std::memcpy(b->h_tab, b->tab.data(), sizeof(BSeries) * (size_t)nseries);
    SSA_TRY_HIP(hipMemcpyAsync(b->ws, b->h_tab, sizeof(BSeries) * (size_t)nseries, hipMemcpyHostToDevice, st));
    SSA_TRY_HIP(hipEventRecord(b->tab_done, st));
    SSA_TRY_HIP(launch_fill_zero(reinterpret_cast<double*>(b->ws + b->t_ndone), 1, st));

    BatchArgs a{};
    a.nseries = nseries;
    a.list = nullptr;
    a.tab = reinterpret_cast<const BSeries*>(b->ws);
    a.ws = b->ws;
    a.ndone = reinterpret_cast<unsigned*>(b->ws + b->t_ndone);
    a.done_flags = nullptr;
    a.check_every = b->cfg.check_every;
    a.onesided = b->cfg.onesided;
    a.tol = b->cfg.tol;

    int kmin = b->tab[0].k, maxcap = 0;
    std::set<int> caps;
    for (const BSeries& t : b->tab) {
        kmin = std::min(kmin, t.k);
        maxcap = std::max(maxcap, t.dcap);
        caps.insert(t.dcap);
    }
    SSA_TRY_HIP(timed(b, SSA_BPROF_INIT, [&] { return launch_batch_init(a, st); }));
    // Lanczos steps in lockstep (every series starts at step 1).  The
    // finished-series count of one check is read while the GPU runs the steps
    // enqueued after it, so the host never waits on the GPU; once every series
    // is finished, the steps already enqueued find nothing left to do.
    int pend = -1, cur = 0;
    for (int j = 1; j <= maxcap + 1; ++j) {
        const int jj = j - 1;
        SSA_TRY_HIP(timed(b, SSA_BPROF_CONV, [&] { return launch_batch_conv(a, 0, st); }));
        SSA_TRY_HIP(timed(b, SSA_BPROF_CGS, [&] { return launch_batch_cgs(a, 0, st); }));
        bool stop = false;
        if (jj >= kmin && (jj % b->cfg.check_every == 0 || caps.count(jj))) {
            SSA_TRY_HIP(timed(b, SSA_BPROF_CHECK, [&] { return launch_batch_check(a, st); }));
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
        SSA_TRY_HIP(timed(b, SSA_BPROF_CONV, [&] { return launch_batch_conv(a, 1, st); }));
        SSA_TRY_HIP(timed(b, SSA_BPROF_CGS, [&] { return launch_batch_cgs(a, 1, st); }));
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

// ===========================================================================
// continuous-batching server: requests join and leave between ticks

namespace {

struct Request {
    long long id;
    unsigned long long key;
    const double* f;
    long long N, L;
    int k;
    double* sigma;
    float* U;
    float* V;
    float* recon;
    int* info;
    ssa_plan plan = nullptr;  // long requests: the single-series plan, sized at submission
    size_t bytes = 0;         // long requests: its workspace bytes
};

// First-fit allocator of byte ranges of the region pool (256-byte multiples).
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    void init(size_t base, size_t bytes) {
        size = bytes;
        free_.clear();
        if (bytes) free_[base] = bytes;
    }
    bool alloc(size_t bytes, size_t* at) {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *at = it->first;
            const size_t rest = it->second - bytes;
            const size_t off = it->first + bytes;
            free_.erase(it);
            if (rest) free_[off] = rest;
            return true;
        }
        return false;
    }
    void release(size_t at, size_t bytes) {
        bytes = align_up(bytes, 256);
        auto it = free_.emplace(at, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto& kv : free_) s += kv.second;
        return s;
    }
};

enum SlotState { kFree = 0, kActive = 1, kFinalizing = 2 };

// A request longer than the batched engine takes, solved on a plan bound to a pool region.
struct LongSlot {
    int state = kFree;
    Request req{};
    size_t reg = 0, bytes = 0;
    hipStream_t stream = nullptr;
    hipEvent_t fin_ev = nullptr;  // its Ritz triples and Hankelization have run
    int* h_info = nullptr;        // pinned: the info ints, staged for the device copy
    ssa::PlanHost host;           // lent to each plan the slot runs (nothing allocated per request)
    int stub_left = 0;
};

// start-vector seed of a long request: a function of the server seed and the request key
unsigned long long long_seed(unsigned long long seed, unsigned long long key) {
    const unsigned long long z = seed ^ (key * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL);
    return z ? z : 1ULL;
}

}  // namespace

struct ssa_server_s {
    EngineCfg cfg;
    ssa_opts opts{};  // as given at creation (the long requests' plans use it)
    int slots;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    size_t o_tab, o_flags, o_lists;  // table, done flags, launch lists (device)
    Pool pool;
    std::deque<Request> queue;         // both classes, in arrival order
    std::vector<int> state;            // SlotState per slot
    std::vector<Request> req;          // request per slot
    std::vector<size_t> reg, reg_bytes;
    BSeries* h_tab = nullptr;          // pinned: table staging (one entry per slot)
    int* h_flags = nullptr;            // pinned: done flags read back after each tick
    int* h_lists = nullptr;            // pinned: launch lists (set-up | active | finalize)
    long long ticks = 0;
    long long n_long_max = 0;          // 0: long requests are not served
    std::vector<LongSlot> lslot;
    int lrr = 0;                       // round-robin position among the long slots
    int stub = 0;                      // stub executor: no device work, requests take stub_ticks ticks
    int stub_ticks = 0;
    std::vector<int> stub_left;        // short slots, stub executor
};

namespace {

void destroy_long(ssa_server v) {
    for (LongSlot& ls : v->lslot) {
        if (ls.stream) (void)hipStreamSynchronize(ls.stream);
        if (ls.req.plan) ssa_plan_destroy(ls.req.plan);
        if (ls.fin_ev) (void)hipEventDestroy(ls.fin_ev);
        if (ls.stream) (void)hipStreamDestroy(ls.stream);
        if (ls.h_info) (void)hipHostFree(ls.h_info);
        if (ls.host.h_scal) ssa::host_free(ls.host);
    }
    v->lslot.clear();
}

// Ritz triples, info and Hankelization of a long request whose stopping test held.
int finish_long(ssa_server v, LongSlot& ls) {
    const Request& r = ls.req;
    ssa_info info{};
    const int rc = ssa::run_finish(r.plan, r.sigma, r.U, r.V, &info);
    int* hi = ls.h_info;
    if (rc == SSA_ENONFINITE) {
        hi[0] = 0;
        hi[1] = -1;  // the series holds NaN or Inf: no triples
        hi[2] = hi[3] = 0;
    } else if (rc < 0) {
        return rc;
    } else {
        hi[0] = info.steps;
        hi[1] = info.converged;
        hi[2] = info.restarts;
        hi[3] = info.dgks_passes;
        if (r.recon) {  // every triple alone, like the batched requests
            std::vector<int> offs(r.k + 1), mem(r.k);
            for (int i = 0; i <= r.k; ++i) offs[i] = i;
            for (int i = 0; i < r.k; ++i) mem[i] = i;
            const int rr = ssa_reconstruct(r.plan, r.sigma, r.U, r.V, r.k, offs.data(), mem.data(), r.k, r.recon);
            if (rr != SSA_OK) return rr;
        }
    }
    if (r.info && hipMemcpyAsync(r.info, hi, sizeof(int) * 4, hipMemcpyHostToDevice, ls.stream) != hipSuccess)
        return SSA_EDEVICE;
    if (hipEventRecord(ls.fin_ev, ls.stream) != hipSuccess) return SSA_EDEVICE;
    return SSA_OK;
}

// One check interval more for active long requests whose previous interval has run (its
// stopping test included: the interval then waits on nothing), and the finish for each
// whose test held; at most `limit` of them, round robin.  *did: something was enqueued.
int advance_long(ssa_server v, bool* did, int limit) {
    *did = false;
    const int n = (int)v->lslot.size();
    for (int t = 0; t < n && limit > 0; ++t) {
        LongSlot& ls = v->lslot[(v->lrr + t) % n];
        if (ls.state != kActive) continue;
        ssa_plan pl = ls.req.plan;
        if (!ssa::run_idle(pl)) continue;  // still working through its previous interval
        if (!ssa::run_stopped(pl)) {
            const int rc = ssa::run_advance(pl, v->cfg.check_every);
            if (rc != SSA_OK) return rc;
            *did = true;
        }
        if (ssa::run_stopped(pl)) {
            const int rc = finish_long(v, ls);
            if (rc != SSA_OK) return rc;
            ls.state = kFinalizing;
            *did = true;
        }
        v->lrr = (v->lrr + t + 1) % n;
        --limit;
    }
    return SSA_OK;
}

int server_create(long long n_max, int k_max, int slots, const ssa_opts* opts, void* workspace_dev, size_t bytes,
                  void* hip_stream, int stub, int stub_ticks, ssa_server* out) {
    if (!out) return SSA_EINVAL;
    *out = nullptr;
    if (!cfg_valid(n_max, k_max, opts) || slots < 1) return SSA_EINVAL;
    if (!stub && (!workspace_dev || reinterpret_cast<uintptr_t>(workspace_dev) % 256)) return SSA_EINVAL;
    if (stub && stub_ticks < 1) return SSA_EINVAL;
    ssa_server v = new (std::nothrow) ssa_server_s();
    if (!v) return SSA_EINVAL;
    v->cfg = make_cfg(n_max, k_max, opts);
    if (opts) v->opts = *opts;
    v->slots = slots;
    v->o_tab = 0;
    v->o_flags = align_up(sizeof(BSeries) * (size_t)slots, 256);
    v->o_lists = v->o_flags + align_up(sizeof(int) * (size_t)slots, 256);
    const size_t head = v->o_lists + align_up(sizeof(int) * 3 * (size_t)slots, 256);
    if (bytes <= head) {
        delete v;
        return SSA_ENOMEM;
    }
    v->ws = static_cast<char*>(workspace_dev);
    v->ws_bytes = bytes;
    v->stream = static_cast<hipStream_t>(hip_stream);
    v->pool.init(head, (bytes - head) / 256 * 256);
    v->state.assign(slots, kFree);
    v->req.assign(slots, Request{});
    v->reg.assign(slots, 0);
    v->reg_bytes.assign(slots, 0);
    v->stub = stub;
    v->stub_ticks = stub_ticks;
    v->stub_left.assign(slots, 0);
    *out = v;
    return SSA_OK;
}

// Workspace bytes and host plan of a long request (N above the batched engine's n_max).
int long_plan(ssa_server v, long long N, long long L, int k, unsigned long long key, ssa_plan* plan,
              size_t* bytes) {
    if (v->n_long_max == 0 || N > v->n_long_max || N <= v->cfg.n_max) return SSA_EINVAL;
    if (L <= 1 || L >= N || k < 1 || k > v->cfg.k_max || k > std::min(L, N - L + 1)) return SSA_EINVAL;
    ssa_opts o = v->opts;
    o.seed = long_seed(v->cfg.seed, key);
    o.restart_keep = 0;
    o.fft_m1 = o.fft_cb = 0;
    o.fft_mp = 0;
    return ssa_embed_plan(N, L, k, &o, bytes, plan);
}

}  // namespace

extern "C" {

int ssa_server_create(long long n_max, int k_max, int slots, const ssa_opts* opts, void* workspace_dev, size_t bytes,
                      void* hip_stream, ssa_server* out) {
    return server_create(n_max, k_max, slots, opts, workspace_dev, bytes, hip_stream, 0, 0, out);
}

int ssa_server_create_stub(long long n_max, int k_max, int slots, const ssa_opts* opts, size_t pool_bytes,
                           int ticks, ssa_server* out) {
    return server_create(n_max, k_max, slots, opts, nullptr, pool_bytes, nullptr, 1, ticks, out);
}

int ssa_server_enable_long(ssa_server v, long long n_long_max, int long_slots) {
    if (!v || long_slots < 1 || n_long_max <= v->cfg.n_max || n_long_max > (1LL << 24)) return SSA_EINVAL;
    if (!v->lslot.empty()) return SSA_ESTATE;
    v->lslot.resize(long_slots);
    v->n_long_max = n_long_max;
    if (v->stub) return SSA_OK;
    for (LongSlot& ls : v->lslot) {
        if (hipStreamCreateWithFlags(&ls.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ls.fin_ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&ls.h_info, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess ||
            ssa::host_alloc_for(ls.host, v->cfg.k_max, &v->opts) != SSA_OK) {
            destroy_long(v);
            v->n_long_max = 0;
            return SSA_EDEVICE;
        }
    }
    return SSA_OK;
}

int ssa_server_request_bytes(ssa_server v, long long N, long long L, int k, size_t* bytes) {
    if (!v || !bytes) return SSA_EINVAL;
    if (N > v->cfg.n_max) {
        ssa_plan pl = nullptr;
        const int rc = long_plan(v, N, L, k, 0, &pl, bytes);
        if (pl) ssa_plan_destroy(pl);
        if (rc == SSA_OK) *bytes = align_up(*bytes, 256);
        return rc;
    }
    BSeries t;
    const size_t b = layout_series(v->cfg, N, L, k, 0, t);
    if (b == 0) return SSA_EINVAL;
    *bytes = b;
    return SSA_OK;
}

int ssa_server_submit(ssa_server v, long long id, unsigned long long key, const double* series_dev, long long N,
                      long long L, int k, double* sigma_dev, float* U_dev, float* V_dev, float* recon_dev,
                      int* info_dev) {
    if (!v || !series_dev || !sigma_dev || !U_dev || !V_dev) return SSA_EINVAL;
    Request r{id, key, series_dev, N, L, k, sigma_dev, U_dev, V_dev, recon_dev, info_dev};
    if (N > v->cfg.n_max) {
        size_t bytes = 0;
        ssa_plan pl = nullptr;
        const int rc = long_plan(v, N, L, k, key, &pl, &bytes);
        if (rc != SSA_OK) {
            if (pl) ssa_plan_destroy(pl);
            return rc;
        }
        if (align_up(bytes, 256) > v->pool.size) {  // could never be admitted
            ssa_plan_destroy(pl);
            return SSA_ENOMEM;
        }
        r.plan = pl;
        r.bytes = bytes;
    } else {
        BSeries t;
        const size_t bytes = layout_series(v->cfg, N, L, k, key, t);
        if (bytes == 0) return SSA_EINVAL;
        if (bytes > v->pool.size) return SSA_ENOMEM;
    }
    v->queue.push_back(r);
    return SSA_OK;
}

int ssa_server_step(ssa_server v, long long* completed, int max_completed, int* ncompleted) {
    if (!v || !ncompleted || max_completed < 0 || (max_completed > 0 && !completed)) return SSA_EINVAL;
    *ncompleted = 0;
    hipStream_t st = v->stream;
    if (!v->h_tab) {  // staging, allocated at the first tick (pinned unless the executor is a stub)
        if (v->stub) {
            v->h_tab = new BSeries[v->slots];
            v->h_flags = new int[v->slots];
            v->h_lists = new int[3 * (size_t)v->slots];
        } else if (hipHostMalloc((void**)&v->h_tab, sizeof(BSeries) * (size_t)v->slots, hipHostMallocDefault) !=
                       hipSuccess ||
                   hipHostMalloc((void**)&v->h_flags, sizeof(int) * (size_t)v->slots, hipHostMallocDefault) !=
                       hipSuccess ||
                   hipHostMalloc((void**)&v->h_lists, sizeof(int) * 3 * (size_t)v->slots, hipHostMallocDefault) !=
                       hipSuccess) {
            return SSA_EDEVICE;
        }
        std::memset(v->h_flags, 0, sizeof(int) * (size_t)v->slots);
    }
    // 1. requests finalized in the previous tick are complete (every tick ends with the
    //    batched stream synchronized; a long request when its own stream has run its finish)
    for (int s = 0; s < v->slots; ++s) {
        if (v->state[s] != kFinalizing) continue;
        if (*ncompleted >= max_completed) break;  // the rest are reported next time
        completed[(*ncompleted)++] = v->req[s].id;
        v->pool.release(v->reg[s], v->reg_bytes[s]);
        v->state[s] = kFree;
    }
    for (LongSlot& ls : v->lslot) {
        if (ls.state != kFinalizing) continue;
        if (*ncompleted >= max_completed) break;
        if (!v->stub && hipEventQuery(ls.fin_ev) != hipSuccess) continue;
        completed[(*ncompleted)++] = ls.req.id;
        v->pool.release(ls.reg, ls.bytes);
        ssa_plan_destroy(ls.req.plan);
        ls.req.plan = nullptr;
        ls.state = kFree;
    }
    // 2. long requests: one check interval more for each whose last one has run; the
    //    finish (Ritz triples, Hankelization) for each whose stopping test held: done
    //    while the batched step below runs (stub: counted down here)
    if (v->stub)
        for (LongSlot& ls : v->lslot)
            if (ls.state == kActive && --ls.stub_left <= 0) ls.state = kFinalizing;
    BatchArgs a{};
    a.tab = reinterpret_cast<const BSeries*>(v->ws + v->o_tab);
    a.ws = v->ws;
    a.ndone = nullptr;
    a.done_flags = reinterpret_cast<int*>(v->ws + v->o_flags);
    a.check_every = v->cfg.check_every;
    a.onesided = v->cfg.onesided;
    a.tol = v->cfg.tol;
    int* d_lists = reinterpret_cast<int*>(v->ws + v->o_lists);
    int* l_init = v->h_lists;
    int* l_act = v->h_lists + v->slots;
    int* l_fin = v->h_lists + 2 * v->slots;
    int n_init = 0, n_act = 0, n_fin = 0;
    // 3. batched series the previous tick's stopping test finished: Ritz triples and Hankelization
    for (int s = 0; s < v->slots; ++s)
        if (v->state[s] == kActive && v->h_flags[s]) l_fin[n_fin++] = s;
    // 4. admission in arrival order: a request whose class has no free slot lets later
    //    requests of the other class pass; one that the pool cannot hold stops admission
    //    (nothing overtakes a request waiting for memory)
    for (auto it = v->queue.begin(); it != v->queue.end();) {
        const Request& r = *it;
        if (r.plan) {
            int ls_i = -1;
            for (int c = 0; c < (int)v->lslot.size(); ++c)
                if (v->lslot[c].state == kFree) {
                    ls_i = c;
                    break;
                }
            if (ls_i < 0) {
                ++it;
                continue;
            }
            size_t at = 0;
            if (!v->pool.alloc(r.bytes, &at)) break;
            LongSlot& ls = v->lslot[ls_i];
            ls.req = r;
            ls.reg = at;
            ls.bytes = r.bytes;
            ls.state = kActive;
            ls.stub_left = v->stub_ticks;
            if (!v->stub) {
                int rc = ssa::plan_lend_host(r.plan, ls.host);
                if (rc == SSA_OK) rc = ssa_plan_bind(r.plan, v->ws + at, align_up(r.bytes, 256), ls.stream);
                if (rc == SSA_OK) rc = ssa::run_begin(r.plan, r.f, r.k);
                if (rc == SSA_OK) rc = ssa::run_advance(r.plan, v->cfg.check_every);
                if (rc != SSA_OK) return rc;
            }
        } else {
            int s = -1;
            for (int c = 0; c < v->slots; ++c)
                if (v->state[c] == kFree) {
                    s = c;
                    break;
                }
            if (s < 0) {
                ++it;
                continue;
            }
            BSeries t;
            const size_t bytes = layout_series(v->cfg, r.N, r.L, r.k, r.key, t);
            size_t at = 0;
            if (!v->pool.alloc(bytes, &at)) break;
            t.reg = (long long)at;
            t.f = r.f;
            t.sigma = r.sigma;
            t.U = r.U;
            t.V = r.V;
            t.recon = r.recon;
            t.info = r.info;
            v->h_tab[s] = t;
            if (!v->stub)
                SSA_TRY_HIP(hipMemcpyAsync(v->ws + v->o_tab + sizeof(BSeries) * (size_t)s, &v->h_tab[s],
                                           sizeof(BSeries), hipMemcpyHostToDevice, st));
            v->req[s] = r;
            v->reg[s] = at;
            v->reg_bytes[s] = bytes;
            v->state[s] = kActive;
            v->h_flags[s] = 0;
            v->stub_left[s] = v->stub_ticks;
            l_init[n_init++] = s;
        }
        it = v->queue.erase(it);
    }
    for (int s = 0; s < v->slots; ++s)
        if (v->state[s] == kActive && !v->h_flags[s]) l_act[n_act++] = s;
    for (int i = 0; i < n_fin; ++i) v->state[l_fin[i]] = kFinalizing;
    if (v->stub) {  // no device work: a batched request's test holds after stub_ticks ticks
        for (int i = 0; i < n_act; ++i) {
            const int s = l_act[i];
            if (--v->stub_left[s] <= 0) v->h_flags[s] = 1;
        }
        ++v->ticks;
        return SSA_OK;
    }
    SSA_TRY_HIP(hipMemcpyAsync(d_lists, v->h_lists, sizeof(int) * 3 * (size_t)v->slots, hipMemcpyHostToDevice, st));
    if (n_fin) {
        a.list = d_lists + 2 * v->slots;
        a.nseries = n_fin;
        SSA_TRY_HIP(launch_batch_ritz(a, st));
        SSA_TRY_HIP(launch_batch_hankel(a, st));
    }
    if (n_init) {
        a.list = d_lists;
        a.nseries = n_init;
        SSA_TRY_HIP(launch_batch_init(a, st));
    }
    // 5. one Lanczos step of every active batched series; the stopping test runs where it is due
    if (n_act) {
        a.list = d_lists + v->slots;
        a.nseries = n_act;
        SSA_TRY_HIP(launch_batch_conv(a, 0, st));
        SSA_TRY_HIP(launch_batch_cgs(a, 0, st));
        SSA_TRY_HIP(launch_batch_check(a, st));
        SSA_TRY_HIP(launch_batch_conv(a, 1, st));
        SSA_TRY_HIP(launch_batch_cgs(a, 1, st));
    }
    SSA_TRY_HIP(hipMemcpyAsync(v->h_flags, a.done_flags, sizeof(int) * (size_t)v->slots, hipMemcpyDeviceToHost, st));
    // The tick ends when the batched stream has run.  Meanwhile the long requests keep
    // their streams fed, one at a time so that the end of the batched step is seen soon
    // (each advance is one whole check interval, so the sequence of tests, and with it
    // the result, does not depend on timing).  With no batched work every long request
    // gets its interval.
    const bool batched = n_act + n_fin + n_init > 0;
    for (;;) {
        const hipError_t q = hipStreamQuery(st);
        if (q != hipSuccess && q != hipErrorNotReady) return SSA_EDEVICE;
        bool did = false;
        if (q == hipSuccess && batched) break;
        const int rc = advance_long(v, &did, q == hipSuccess ? (int)v->lslot.size() : 1);
        if (rc != SSA_OK) return rc;
        if (q == hipSuccess) break;
        if (!did) std::this_thread::yield();
    }
    ++v->ticks;
    return SSA_OK;
}

int ssa_server_status(ssa_server v, int* queued, int* active, int* finalizing, size_t* pool_free_bytes) {
    if (!v) return SSA_EINVAL;
    int na = 0, nf = 0;
    for (int s = 0; s < v->slots; ++s) {
        na += v->state[s] == kActive;
        nf += v->state[s] == kFinalizing;
    }
    for (const LongSlot& ls : v->lslot) {
        na += ls.state == kActive;
        nf += ls.state == kFinalizing;
    }
    if (queued) *queued = (int)v->queue.size();
    if (active) *active = na;
    if (finalizing) *finalizing = nf;
    if (pool_free_bytes) *pool_free_bytes = v->pool.free_bytes();
    return SSA_OK;
}

void ssa_server_destroy(ssa_server v) {
    if (!v) return;
    if (!v->stub && v->h_tab) (void)hipStreamSynchronize(v->stream);
    destroy_long(v);
    for (Request& r : v->queue)
        if (r.plan) ssa_plan_destroy(r.plan);
    if (v->stub) {
        delete[] v->h_tab;
        delete[] v->h_flags;
        delete[] v->h_lists;
    } else {
        if (v->h_tab) (void)hipHostFree(v->h_tab);
        if (v->h_flags) (void)hipHostFree(v->h_flags);
        if (v->h_lists) (void)hipHostFree(v->h_lists);
    }
    delete v;
}

}  // extern "C"

static_assert(sizeof(BSeries) % 8 == 0, "series table entries must keep 8-byte alignment");
static_assert(batch::kMaxMp <= batch::kEpt * batch::kFftThreads, "in-LDS FFT needs M' <= EPT * threads");
