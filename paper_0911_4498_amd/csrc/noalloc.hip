// noalloc.hip -- ssa_matvec_static: the trajectory-matrix product of ssa_matvec
// (Algorithms 2 and 3 of Sec. 4.3) for callers that cannot allocate device memory
// or bind a workspace (code under HIP graph capture, tight serving loops).
//
// Every intermediate of the product -- the twiddle tables, the spectral operator
// of the series (Algorithm 2, steps 1-2) and the two FFT buffers -- lives in the
// file-scope array `scratch` below, one copy per GPU, held until the process
// ends.  The array's name is a host-side stand-in, not a device address: host
// code uses only the pointer hipGetSymbolAddress returns for the current device.
// The kernels and the FFT schedule are those of a plan made by ssa_embed_plan
// without options, so the result has the same bits as ssa_embed + ssa_matvec.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ssa.h"
#include "ssa_internal.h"

using namespace ssa;

namespace {

constexpr long long kStaticMaxN = 1LL << 20;  // longest series: M' <= 2^19
constexpr int kMaxDevices = 64;
// AB 16 M' + T1, T2 8 M' each (M' <= 2^19), plus the twiddle tables (M1, M2 <= 4096,
// two-level tables of <= 2^10 + 2^9 entries), each region 256-byte aligned.
constexpr size_t kStaticBytes = (size_t)32 * (1u << 19) + (size_t)256 * 1024;

__device__ __align__(256) char scratch[kStaticBytes];

std::mutex g_init_mu;
void* g_dev_scratch[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct StaticLayout {
    size_t ab, tw1, tw2, twlo, twhi, t1, t2, bytes;
};

StaticLayout static_layout(const ConvGeom& g) {
    StaticLayout l{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o = align256(o + b);
        return r;
    };
    const long long S = 1LL << g.tw_shift;
    l.ab = take(sizeof(float4) * (size_t)g.Mp);
    l.tw1 = take(sizeof(float2) * (size_t)g.M1);
    l.tw2 = take(sizeof(float2) * (size_t)g.M2);
    l.twlo = take(sizeof(float2) * (size_t)S);
    l.twhi = take(sizeof(float2) * (size_t)((g.Mp + S - 1) / S));
    l.t1 = take(sizeof(float2) * (size_t)g.Mp);
    l.t2 = take(sizeof(float2) * (size_t)g.Mp);
    l.bytes = o;
    return l;
}

// The device address of this GPU's copy of `scratch`, looked up once per device
// with that device current; nullptr on failure.
char* device_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!g_dev_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_dev_scratch[dev] = ptr;
    }
    return static_cast<char*>(g_dev_scratch[dev]);
}

}  // namespace

extern "C" {

int ssa_matvec_static(const double* series_dev, long long N, long long L, int transpose, const float* x_dev,
                      float* y_dev, void* hip_stream) {
    if (!series_dev || !x_dev || !y_dev) return SSA_EINVAL;
    if (N <= 2 || L <= 1 || L >= N) return SSA_EINVAL;
    if (N > kStaticMaxN) return SSA_ENOMEM;
    ConvGeom g{};
    if (!auto_geometry(N, &g)) return SSA_EINVAL;
    const StaticLayout lay = static_layout(g);
    if (lay.bytes > kStaticBytes) return SSA_ENOMEM;
    if (kernel_attributes_once() != hipSuccess) return SSA_EDEVICE;
    char* base = device_scratch();
    if (!base) return SSA_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    g.tw1 = reinterpret_cast<const float2*>(base + lay.tw1);
    g.tw2 = reinterpret_cast<const float2*>(base + lay.tw2);
    g.tw_lo = reinterpret_cast<const float2*>(base + lay.twlo);
    g.tw_hi = reinterpret_cast<const float2*>(base + lay.twhi);
    float2* T1 = reinterpret_cast<float2*>(base + lay.t1);
    float2* T2 = reinterpret_cast<float2*>(base + lay.t2);
    float4* AB = reinterpret_cast<float4*>(base + lay.ab);
    if (launch_tables(g, const_cast<float2*>(g.tw1), const_cast<float2*>(g.tw2), const_cast<float2*>(g.tw_lo),
                      const_cast<float2*>(g.tw_hi), s) != hipSuccess)
        return SSA_EDEVICE;
    // Algorithm 2, steps 1-2: the operator of the series
    P1In ser{};
    ser.f = series_dev;
    ser.N = N;
    if (launch_pass1(g, IN_SERIES, ser, 1, T1, s) != hipSuccess) return SSA_EDEVICE;
    if (launch_pass2_embed(g, T1, AB, s) != hipSuccess) return SSA_EDEVICE;
    // the product: X x takes K entries and gives L, X^T x takes L and gives K
    const long long K = N - L + 1;
    const long long n_in = transpose ? L : K;
    P1In in{};
    in.x = x_dev;
    in.n_in = n_in;
    if (launch_pass1(g, IN_REV, in, 1, T1, s) != hipSuccess) return SSA_EDEVICE;
    if (launch_pass2_matvec(g, AB, T1, T2, s) != hipSuccess) return SSA_EDEVICE;
    P3Out o{};
    o.out = y_dev;
    o.n_in = n_in;
    o.n_out = N + 1 - n_in;
    if (launch_pass3(g, OUT_SLICE, T2, o, 1, s) != hipSuccess) return SSA_EDEVICE;
    return SSA_OK;
}

}  // extern "C"
