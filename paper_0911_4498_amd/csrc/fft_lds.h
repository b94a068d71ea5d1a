// fft_lds.h -- mixed-radix complex FFTs staged in LDS (gfx950, wave64).
//
// The DFT of Sec. 4.1 (forward kernel e^{-2 pi i k l / n}, inverse with
// e^{+2 pi i k l / n} and no 1/n factor -- callers fold the scale into the
// spectral operator).  Each transform is a Stockham autosort sequence of
// radix-R stages (R in {2,3,4,5,7,8}), so the output is in natural order
// without a bit-reversal pass.  One workgroup runs `nseq` independent
// transforms of length n that sit in LDS at buf + s*sstride.  A stage reads
// every butterfly's inputs into registers, synchronizes, and writes the
// outputs back in place, so only one LDS buffer is needed.
#pragma once
#include <hip/hip_runtime.h>

namespace ssa {

constexpr int kMaxStages = 16;

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also makes the
// workgroup's earlier global stores visible to it, which on this GPU waits for every
// store in flight to complete; the kernels that use this barrier never read global
// memory that another thread of the workgroup wrote in the same launch.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct FftStages {
    int n;
    int nstages;
    int radix[kMaxStages];
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// a * e^{DIR i pi/2}: forward (DIR=-1) multiplies by -i, inverse by +i.
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int R>
struct OddRadix;
template <>
struct OddRadix<3> {
    static __device__ __forceinline__ float c(int q) { return -0.5f; }
    static __device__ __forceinline__ float s(int q) {
        return q == 1 ? 0.866025403784438647f : -0.866025403784438647f;
    }
};
template <>
struct OddRadix<5> {
    static __device__ __forceinline__ float c(int q) {
        return (q == 1 || q == 4) ? 0.309016994374947424f : -0.809016994374947424f;
    }
    static __device__ __forceinline__ float s(int q) {
        switch (q) {
            case 1: return 0.951056516295153572f;
            case 2: return 0.587785252292473129f;
            case 3: return -0.587785252292473129f;
            default: return -0.951056516295153572f;
        }
    }
};
template <>
struct OddRadix<7> {
    static __device__ __forceinline__ float c(int q) {
        switch (q) {
            case 1: case 6: return 0.623489801858733531f;
            case 2: case 5: return -0.222520933956314404f;
            default: return -0.900968867902419126f;
        }
    }
    static __device__ __forceinline__ float s(int q) {
        switch (q) {
            case 1: return 0.781831482468029809f;
            case 2: return 0.974927912181823607f;
            case 3: return 0.433883739117558120f;
            case 4: return -0.433883739117558120f;
            case 5: return -0.974927912181823607f;
            default: return -0.781831482468029809f;
        }
    }
};

// In-register DFT of length R: y_m = sum_r x_r e^{DIR 2 pi i r m / R}.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
    if constexpr (R == 2) {
        float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 4) {
        float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
        float2 t2 = cadd(x[1], x[3]), t3 = rot90<DIR>(csub(x[1], x[3]));
        x[0] = cadd(t0, t2);
        x[2] = csub(t0, t2);
        x[1] = cadd(t1, t3);
        x[3] = csub(t1, t3);
    } else if constexpr (R == 8) {
        float2 e[4] = {x[0], x[2], x[4], x[6]};
        float2 o[4] = {x[1], x[3], x[5], x[7]};
        dft<4, DIR>(e);
        dft<4, DIR>(o);
        const float h = 0.707106781186547524f;
        float2 o1 = cscale(cadd(o[1], rot90<DIR>(o[1])), h);
        float2 o2 = rot90<DIR>(o[2]);
        float2 o3 = cscale(csub(rot90<DIR>(o[3]), o[3]), h);
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[5] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[6] = csub(e[2], o2);
        x[3] = cadd(e[3], o3);
        x[7] = csub(e[3], o3);
    } else {
        // odd R: pair r with R - r (cosine and sine parts)
        constexpr int H = (R - 1) / 2;
        float2 a[H], b[H];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            a[r - 1] = cadd(x[r], x[R - r]);
            b[r - 1] = rot90<DIR>(csub(x[r], x[R - r]));
        }
        float2 y[R];
        float2 s0 = x[0];
#pragma unroll
        for (int r = 0; r < H; ++r) s0 = cadd(s0, a[r]);
        y[0] = s0;
#pragma unroll
        for (int m = 1; m < R; ++m) {
            float2 acc = x[0];
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const int q = (r * m) % R;
                acc.x += a[r - 1].x * OddRadix<R>::c(q) + b[r - 1].x * OddRadix<R>::s(q);
                acc.y += a[r - 1].y * OddRadix<R>::c(q) + b[r - 1].y * OddRadix<R>::s(q);
            }
            y[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < R; ++m) x[m] = y[m];
    }
}

// Twiddle sources: W(t) = e^{-2 pi i t / n}.
struct TableTw {  // full table of n entries
    const float2* tw;
    __device__ __forceinline__ float2 operator()(int t) const { return tw[t]; }
};
struct TwoLevelTw {  // W(t) = hi[t >> shift] * lo[t & mask]; two tables of ~sqrt(n) entries
    const float2* hi;
    const float2* lo;
    int shift;
    __device__ __forceinline__ float2 operator()(int t) const {
        const float2 a = hi[t >> shift], b = lo[t & ((1 << shift) - 1)];
        return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
    }
};

// W(t) for t < n from a table of the first n/4 entries (n divisible by 4), with
// W(t + n/4) = -i W(t): a quarter of the LDS of the full table.
struct QuarterTableTw {
    const float2* tw;
    int quarter;  // n / 4
    __device__ __forceinline__ float2 operator()(int t) const {
        const int q = (t >= quarter) + (t >= 2 * quarter) + (t >= 3 * quarter);
        const float2 w = tw[t - q * quarter];
        switch (q) {
            case 0: return w;
            case 1: return make_float2(w.y, -w.x);
            case 2: return make_float2(-w.x, -w.y);
            default: return make_float2(-w.y, w.x);
        }
    }
};

// Ordering of LDS accesses within one wave (the wave's LDS instructions complete in issue
// order; this keeps the compiler from moving them across it).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// One Stockham stage of radix R over nseq sequences of length n.  WAVE: the transform
// belongs to one wave (tid = lane, nthr = 64), whose stages need no workgroup barrier.
// p = product of the radices of earlier stages; tw(t) = e^{-2 pi i t / n}.
template <int R, int DIR, int EPT, typename TW, bool WAVE = false>
__device__ __forceinline__ void fft_stage(float2* buf, int n, int nseq, int sstride, int p,
                                          const TW& tw, int tid, int nthr) {
    constexpr int NB = (EPT + R - 1) / R;
    const int nq = n / R;
    const int nb = nq * nseq;
    const int twstep = n / (p * R);
    float2 v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid + i * nthr;
        if (b < nb) {
            const int s = b / nq;
            const int q = b - s * nq;
            const int k = q % p;
            const float2* src = buf + s * sstride + q;
            float2 x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = src[r * nq];
            if (p > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw(r * k * twstep);
                    if (DIR > 0) w.y = -w.y;
                    x[r] = cmul(x[r], w);
                }
            }
            dft<R, DIR>(x);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = x[r];
        }
    }
    if constexpr (WAVE)
        wave_lds_sync();
    else
        lds_barrier();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid + i * nthr;
        if (b < nb) {
            const int s = b / nq;
            const int q = b - s * nq;
            const int k = q % p;
            float2* dst = buf + s * sstride + (q - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * p] = v[i][r];
        }
    }
    if constexpr (WAVE)
        wave_lds_sync();
    else
        lds_barrier();
}

// Full transform.  Requires n * nseq <= EPT * nthr.  Ends synchronized.
template <int DIR, int EPT, typename TW>
__device__ void lds_fft_tw(float2* buf, const FftStages& st, int nseq, int sstride, const TW& tw,
                           int tid, int nthr) {
    int p = 1;
    for (int s = 0; s < st.nstages; ++s) {
        const int R = st.radix[s];
        switch (R) {
            case 8: fft_stage<8, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
            case 4: fft_stage<4, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
            case 2: fft_stage<2, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
            case 3: fft_stage<3, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
            case 5: fft_stage<5, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
            default: fft_stage<7, DIR, EPT>(buf, st.n, nseq, sstride, p, tw, tid, nthr); break;
        }
        p *= R;
    }
}

template <int DIR, int EPT>
__device__ void lds_fft(float2* buf, const FftStages& st, int nseq, int sstride,
                        const float2* __restrict__ tw, int tid, int nthr) {
    lds_fft_tw<DIR, EPT>(buf, st, nseq, sstride, TableTw{tw}, tid, nthr);
}

// Radix sequences known at compile time.  A kernel instantiated with FftFixed<R...> inlines
// exactly those stages (no run-time radix switch): its code is a fraction of the generic
// one's, which matters when each launch is short and starts with cold instruction caches.
// FftGeneric runs the sequence of the FftStages argument.
struct FftGeneric {
    static constexpr bool kFixed = false;
    static __host__ __device__ bool matches(const FftStages&) { return true; }
};
template <int... R>
struct FftFixed {
    static constexpr bool kFixed = true;
    static constexpr int kLength = (R * ...);
    static __host__ __device__ bool matches(const FftStages& st) {
        constexpr int r[] = {R...};
        if (st.nstages != (int)sizeof...(R)) return false;
        for (int i = 0; i < (int)sizeof...(R); ++i)
            if (st.radix[i] != r[i]) return false;
        return true;
    }
};

template <int DIR, int EPT>
__device__ __forceinline__ void fft_run(FftGeneric, float2* buf, const FftStages& st, int nseq, int sstride,
                                        const float2* __restrict__ tw, int tid, int nthr) {
    lds_fft<DIR, EPT>(buf, st, nseq, sstride, tw, tid, nthr);
}

template <int DIR, int EPT, int... R>
__device__ __forceinline__ void fft_run(FftFixed<R...>, float2* buf, const FftStages&, int nseq, int sstride,
                                        const float2* __restrict__ tw, int tid, int nthr) {
    constexpr int n = (R * ...);  // the length, and with it every stride and twiddle step, is a constant
    int p = 1;
    ((fft_stage<R, DIR, EPT>(buf, n, nseq, sstride, p, TableTw{tw}, tid, nthr), p *= R), ...);
}

// One transform of a fixed length by one wave (lane < 64; at most 4 points per lane, so
// n <= 256), with no workgroup barrier between its stages: the caller synchronizes the
// workgroup before other waves read the result.
template <int DIR, int... R>
__device__ __forceinline__ void fft_run_wave(FftFixed<R...>, float2* buf, const float2* __restrict__ tw, int lane) {
    constexpr int n = (R * ...);
    static_assert(n <= 256, "one wave, four points per lane");
    int p = 1;
    ((fft_stage<R, DIR, 4, TableTw, true>(buf, n, 1, n, p, TableTw{tw}, lane, 64), p *= R), ...);
}

// nseq transforms of a fixed length of at most 256 points, one per wave (nseq <= waves),
// or the workgroup-wide transform otherwise; ends synchronized.
template <int DIR, int EPT, typename F>
__device__ __forceinline__ void fft_run_waves(F f, float2* buf, const FftStages& st, int nseq, int sstride,
                                              const float2* __restrict__ tw, int tid, int nthr) {
    if constexpr (F::kFixed) {
        if constexpr (F::kLength <= 256) {
            if (nseq <= nthr / 64) {
                const int wave = tid >> 6;
                if (wave < nseq) fft_run_wave<DIR>(f, buf + (long long)wave * sstride, tw, tid & 63);
                lds_barrier();
                return;
            }
        }
    }
    fft_run<DIR, EPT>(f, buf, st, nseq, sstride, tw, tid, nthr);
}

// The same with the twiddles from a quarter table (tw holds W(t) for t < n/4).
template <int DIR, int EPT, int... R>
__device__ __forceinline__ void fft_run_quarter(FftFixed<R...>, float2* buf, int nseq, int sstride,
                                                const float2* __restrict__ tw, int tid, int nthr) {
    constexpr int n = (R * ...);
    static_assert(n % 4 == 0, "quarter table needs n divisible by 4");
    const QuarterTableTw q{tw, n / 4};
    int p = 1;
    ((fft_stage<R, DIR, EPT>(buf, n, nseq, sstride, p, q, tid, nthr), p *= R), ...);
}

}  // namespace ssa
