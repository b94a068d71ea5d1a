// kernels.hip -- gfx950 kernels of the fast SSA hot path.
//
//  * FFT convolution passes (Sec. 4, Algorithms 2/3 for X v and X^T u; Sec. 5,
//    Algorithm 4 for rank-1 Hankelization), built on the LDS FFT of fft_lds.h.
//    A real sequence w of length M is packed as z[n] = w[2n] + i w[2n+1]
//    (M' = M/2 complex points).  With Z = DFT_{M'}(z):
//        W(k)      = E(k) + w_M^k O(k),   W(k + M') = E(k) - w_M^k O(k),
//        E(k) = (Z(k) + conj Z(M'-k)) / 2,  O(k) = -i (Z(k) - conj Z(M'-k)) / 2,
//    w_M = e^{-2 pi i / M}.  Every spectral step therefore pairs bin k with
//    bin M'-k; in the transposed layout T[k1][k2] the partner of (k1, k2) is
//    (M1-k1, M2-1-k2) for k1 > 0 and (0, (M2-k2) mod M2) for k1 = 0, so one
//    workgroup of pass 2 owns rows k1 and M1-k1 and needs no exchange.
//  * Classical Gram-Schmidt reorthogonalization (Sec. 3.2.2) split into a
//    projection kernel (FP64 partial inner products), a one-workgroup
//    reduction (coefficients, the new alpha/beta, the DGKS test and the
//    breakdown restart) and an update kernel that writes the normalized
//    Lanczos vector.
//  * Ritz-vector assembly U_{d+1} P and V_d Q (eqs. lbdiagm1/lbdiagm2).
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "ssa_internal.h"

namespace ssa {

thread_local LaunchTiming g_launch_timing;

// ---------------------------------------------------------------------------
// twiddle tables (FP64 angles, rounded once to FP32)

__global__ void k_tables(int M1, int M2, long long Mp, int shift, float2* tw1, float2* tw2,
                         float2* tw_lo, float2* tw_hi) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long S = 1LL << shift;
    const long long nhi = (Mp + S - 1) / S;
    double s, c;
    if (t < M1) {
        sincospi(-2.0 * (double)t / (double)M1, &s, &c);
        tw1[t] = make_float2((float)c, (float)s);
    }
    if (t < M2) {
        sincospi(-2.0 * (double)t / (double)M2, &s, &c);
        tw2[t] = make_float2((float)c, (float)s);
    }
    if (t < S) {
        sincospi(-2.0 * (double)t / (double)Mp, &s, &c);
        tw_lo[t] = make_float2((float)c, (float)s);
    }
    if (t < nhi) {
        sincospi(-2.0 * (double)(t * S) / (double)Mp, &s, &c);
        tw_hi[t] = make_float2((float)c, (float)s);
    }
}

// ---------------------------------------------------------------------------
// pass 1: column FFTs (length M1) of CB adjacent columns, twiddle, store T[k1][n2]

// Position m of the padded coordinates of a width-w array (pitch > 0): its
// compressed index, or -1 in the gap between rows.
__device__ __forceinline__ long long compress_index(long long m, long long pitch, int w) {
    const long long r = m / pitch, c = m - r * pitch;
    return c < w ? r * w + c : -1;
}

template <int MODE>
__device__ __forceinline__ float p1_value(const P1In& a, long long m, int y) {
    if constexpr (MODE == IN_REV) {
        if (m >= a.n_in) return 0.0f;
        long long j = a.n_in - 1 - m;
        if (a.pitch) {
            j = compress_index(j, a.pitch, a.win);
            if (j < 0) return 0.0f;
        }
        return a.x[j];
    } else if constexpr (MODE == IN_SERIES) {
        return m < a.N ? (float)a.f[m] : 0.0f;
    } else {
        const bool isu = y < a.nu;
        if (m >= (isu ? a.lenu : a.lenv)) return 0.0f;
        long long j = m;
        if (a.pitch) {
            j = compress_index(m, a.pitch, isu ? a.wu : a.wv);
            if (j < 0) return 0.0f;
        }
        return isu ? a.U[(long long)y * a.ldu + j] : a.V[(long long)(y - a.nu) * a.ldv + j];
    }
}

// Element m of input y as a position to load: the float (or, for the series, double) at
// *pf / *pd when ok, else the value 0 (pf / pd then point at an element that exists, so
// the load can be issued unconditionally: loads under a branch would be waited for one
// at a time).
template <int MODE>
__device__ __forceinline__ bool p1_where(const P1In& a, long long m, int y, const float*& pf, const double*& pd) {
    if constexpr (MODE == IN_REV) {
        long long j = a.n_in - 1 - m;
        bool ok = m < a.n_in;
        if (a.pitch && ok) {
            j = compress_index(j, a.pitch, a.win);
            ok = j >= 0;
        }
        pf = a.x + (ok ? j : 0);
        return ok;
    } else if constexpr (MODE == IN_SERIES) {
        const bool ok = m < a.N;
        pd = a.f + (ok ? m : 0);
        return ok;
    } else {
        const bool isu = y < a.nu;
        bool ok = m < (isu ? a.lenu : a.lenv);
        long long j = m;
        if (a.pitch && ok) {
            j = compress_index(m, a.pitch, isu ? a.wu : a.wv);
            ok = j >= 0;
        }
        if (!ok) j = 0;
        pf = isu ? a.U + (long long)y * a.ldu + j : a.V + (long long)(y - a.nu) * a.ldv + j;
        return ok;
    }
}

template <int MODE>
__device__ __forceinline__ float p1_load(const float* pf, const double* pd) {
    if constexpr (MODE == IN_SERIES)
        return (float)*pd;
    else
        return *pf;
}

// Threads of a workgroup of the FFT passes whose rows hold more than 2048
// points in total (up to 8192: 8 per thread).  Such a workgroup needs 64-96
// KB of LDS, so it is alone on its CU; the 16 waves are what hides the
// memory latency (256 threads with 32 points each reach a third less).
constexpr int kBigThreads = 1024;


// QTW: the twiddle table in LDS is a quarter table (fixed-radix long rows, F1 = FftFixed), so
// that two workgroups share a CU's LDS.
template <int MODE, int EPT, int NT = 256, typename F1 = FftGeneric, bool QTW = false>
__global__ __launch_bounds__(NT) void k_pass1(ConvGeom g, P1In a, float2* __restrict__ T1) {
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int CB = g.CB, M1 = g.M1, M2 = g.M2, ss = M1 + 1;
    float2* buf = smem;
    float2* tw = smem + CB * ss;
    const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
    const int y = blockIdx.y;
    // the first four elements per thread (two values each) and the first twiddle are
    // loaded before any LDS write; whole waves past the data skip their loads
    const int nz = CB * M1, wave0 = tid & ~63;
    // positions first, then the loads (all unconditional, at clamped positions), then the
    // zeros: branches between them would have each load waited for in turn
    const float* fp[4][2];
    const double* dp[4][2];
    bool okv[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = min(tid + i * nthr, nz - 1);
        const int c = idx % CB, n1 = idx / CB, n2 = min(c0 + c, M2 - 1);
        const long long n = (long long)M2 * n1 + n2;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            fp[i][e] = nullptr;
            dp[i][e] = nullptr;
            okv[i][e] = p1_where<MODE>(a, 2 * n + e, y, fp[i][e], dp[i][e]) && c0 + c < M2 && tid + i * nthr < nz;
        }
    }
    float zr[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 2; ++e) zr[i][e] = p1_load<MODE>(fp[i][e], dp[i][e]);
    float2 zv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) zv[i] = make_float2(okv[i][0] ? zr[i][0] : 0.0f, okv[i][1] ? zr[i][1] : 0.0f);
    (void)wave0;
    const int ntw = QTW ? M1 / 4 : M1;  // entries of the twiddle table
    const float2 tw0 = g.tw1[min(tid, ntw - 1)];
    if (tid < ntw) tw[tid] = tw0;
    for (int t = tid + nthr; t < ntw; t += nthr) tw[t] = g.tw1[t];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = tid + i * nthr;
        if (idx < nz) buf[(idx % CB) * ss + idx / CB] = zv[i];
    }
    for (int idx = tid + 4 * nthr; idx < nz; idx += nthr) {
        const int c = idx % CB, n1 = idx / CB, n2 = c0 + c;
        float2 z = make_float2(0.0f, 0.0f);
        if (n2 < M2) {
            const long long n = (long long)M2 * n1 + n2;
            z.x = p1_value<MODE>(a, 2 * n, y);
            z.y = p1_value<MODE>(a, 2 * n + 1, y);
        }
        buf[c * ss + n1] = z;
    }
    // output twiddles W_{M'}^{n2 k1} of this thread's first kPre stores, fetched before the FFT
    // (not in the 1024-thread instantiations: capped at 128 VGPRs, they would spill)
    constexpr int kPre = NT >= 1024 ? 0 : 4;
    float2 wpre[kPre > 0 ? kPre : 1];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
        // clamped, unconditional loads; the value is used only where idx < CB * M1 and
        // n2 < M2
        const int idx = min(tid + i * nthr, nz - 1);
        const int c = idx % CB, k1 = idx / CB, n2 = min(c0 + c, M2 - 1);
        wpre[i] = twiddle_mp(g, (long long)n2 * k1);
    }
    lds_barrier();
    if constexpr (QTW)
        fft_run_quarter<-1, EPT>(F1{}, buf, CB, ss, tw, tid, nthr);
    else
        fft_run_waves<-1, EPT>(F1{}, buf, g.st1, CB, ss, tw, tid, nthr);
    float2* out = T1 + (long long)y * g.Mp;
    int i = 0;
    for (int idx = tid; idx < CB * M1; idx += nthr, ++i) {
        const int c = idx % CB, k1 = idx / CB, n2 = c0 + c;
        if (n2 < M2) {
            const float2 w = i < kPre ? wpre[i < kPre ? i : 0] : twiddle_mp(g, (long long)n2 * k1);
            out[(long long)k1 * M2 + n2] = cmul(buf[c * ss + k1], w);
        }
    }
}

// ---------------------------------------------------------------------------
// pass 2 helpers: rows a and M1-a, pairs (element, partner)

struct RowPair {
    int a, b, nseq, npairs;
    __device__ RowPair(int a_, int M1, int M2) : a(a_) {
        b = (a == 0) ? 0 : M1 - a;
        const bool two = (a != 0) && (2 * a != M1);
        nseq = two ? 2 : 1;
        npairs = two ? M2 : (a == 0 ? M2 / 2 + 1 : (M2 + 1) / 2);
    }
    // pair p -> (seq, k2) of the element and of its partner
    __device__ void pair(int p, int M2, int& s0, int& e0, int& s1, int& e1) const {
        s0 = 0;
        e0 = p;
        if (nseq == 2) {
            s1 = 1;
            e1 = M2 - 1 - p;
        } else if (a == 0) {
            s1 = 0;
            e1 = (M2 - p) % M2;
        } else {
            s1 = 0;
            e1 = M2 - 1 - p;
        }
    }
    __device__ int row(int s) const { return s ? b : a; }
};

template <int EPT>
__device__ __forceinline__ void load_rows(float2* buf, const float2* __restrict__ T, const RowPair& rp,
                                          int M2, int tid, int nthr) {
    for (int idx = tid; idx < rp.nseq * M2; idx += nthr) {
        const int s = idx / M2, k2 = idx - s * M2;
        buf[idx] = T[(long long)rp.row(s) * M2 + k2];
    }
}

template <int EPT>
__device__ __forceinline__ void store_rows(const float2* buf, float2* __restrict__ T, const RowPair& rp,
                                           int M2, int tid, int nthr) {
    for (int idx = tid; idx < rp.nseq * M2; idx += nthr) {
        const int s = idx / M2, k2 = idx - s * M2;
        T[(long long)rp.row(s) * M2 + k2] = buf[idx];
    }
}

// pass 2 of a trajectory-matrix product: Q(k) = A(k) Z(k) + B(k) conj Z(M'-k)
template <int EPT, int NT = 256, typename F2 = FftGeneric, bool QTW = false>
__global__ __launch_bounds__(NT) void k_pass2_matvec(ConvGeom g, const float4* __restrict__ AB,
                                                      const float2* __restrict__ T1,
                                                      float2* __restrict__ T2) {
    const double stopv = g.stop ? *g.stop : 0.0;  // tested once the row loads are in flight
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int M2 = g.M2;
    float2* buf = smem;
    float2* tw = smem + 2 * M2;
    const RowPair rp(blockIdx.x, g.M1, M2);
    // The first four row elements per thread, the first twiddle and the operator values
    // of the first kPre pairs are loaded (at clamped, in-bounds positions) before any LDS
    // write: a write of a loaded value waits for every load issued before it.
    const int total = rp.nseq * M2;
    const int wave0 = tid & ~63;  // (whole waves past the data skip their loads)
    float2 rv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (wave0 + i * nthr >= total) continue;
        const int idx = min(tid + i * nthr, total - 1);
        const int s = idx / M2, k2 = idx - s * M2;
        rv[i] = T1[(long long)rp.row(s) * M2 + k2];
    }
    const int ntw = QTW ? M2 / 4 : M2;  // entries of the twiddle table
    const float2 tw0 = g.tw2[min(tid, ntw - 1)];
    // (not in the 1024-thread instantiation: capped at 128 VGPRs, it would spill)
    constexpr int kPre = NT >= 1024 ? 0 : 2;
    float4 pre0[kPre > 0 ? kPre : 1], pre1[kPre > 0 ? kPre : 1];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
        if (wave0 + i * nthr >= rp.npairs) continue;
        const int p = min(tid + i * nthr, rp.npairs - 1);
        int s0, e0, s1, e1;
        rp.pair(p, M2, s0, e0, s1, e1);
        pre0[i] = AB[(long long)rp.row(s0) * M2 + e0];
        pre1[i] = AB[(long long)rp.row(s1) * M2 + e1];
    }
    if (tid < ntw) tw[tid] = tw0;
    for (int t = tid + nthr; t < ntw; t += nthr) tw[t] = g.tw2[t];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (tid + i * nthr < total) buf[tid + i * nthr] = rv[i];
    for (int idx = tid + 4 * nthr; idx < total; idx += nthr) {
        const int s = idx / M2, k2 = idx - s * M2;
        buf[idx] = T1[(long long)rp.row(s) * M2 + k2];
    }
    if (stopv != 0.0) return;
    lds_barrier();
    if constexpr (QTW)
        fft_run_quarter<-1, EPT>(F2{}, buf, rp.nseq, M2, tw, tid, nthr);
    else
        fft_run_waves<-1, EPT>(F2{}, buf, g.st2, rp.nseq, M2, tw, tid, nthr);
    int i = 0;
    for (int p = tid; p < rp.npairs; p += nthr, ++i) {
        int s0, e0, s1, e1;
        rp.pair(p, M2, s0, e0, s1, e1);
        const float2 z0 = buf[s0 * M2 + e0], z1 = buf[s1 * M2 + e1];
        const float4 o0 = i < kPre ? pre0[i < kPre ? i : 0] : AB[(long long)rp.row(s0) * M2 + e0];
        const float4 o1 = i < kPre ? pre1[i < kPre ? i : 0] : AB[(long long)rp.row(s1) * M2 + e1];
        const float2 q0 = cadd(cmul(make_float2(o0.x, o0.y), z0), cmul(make_float2(o0.z, o0.w), cconj(z1)));
        const float2 q1 = cadd(cmul(make_float2(o1.x, o1.y), z1), cmul(make_float2(o1.z, o1.w), cconj(z0)));
        buf[s0 * M2 + e0] = q0;
        if (s0 != s1 || e0 != e1) buf[s1 * M2 + e1] = q1;
    }
    lds_barrier();
    if constexpr (QTW)
        fft_run_quarter<1, EPT>(F2{}, buf, rp.nseq, M2, tw, tid, nthr);
    else
        fft_run_waves<1, EPT>(F2{}, buf, g.st2, rp.nseq, M2, tw, tid, nthr);
    store_rows<EPT>(buf, T2, rp, M2, tid, nthr);
}

// E/O split of one packed-real spectrum pair, in FP64.
struct SplitD {
    double er, ei, orr, oi;
};
__device__ __forceinline__ SplitD split_eo(float2 z, float2 zp) {
    // E = (z + conj zp)/2 ; O = -i (z - conj zp)/2
    SplitD s;
    s.er = 0.5 * ((double)z.x + (double)zp.x);
    s.ei = 0.5 * ((double)z.y - (double)zp.y);
    const double dr = (double)z.x - (double)zp.x, di = (double)z.y + (double)zp.y;
    s.orr = 0.5 * di;
    s.oi = -0.5 * dr;
    return s;
}

// Spectral operator of the series (Algorithm 2, steps 1-2, done once).  For a
// real c with full spectrum C, the packed output q = pack(c (*) w) satisfies
//   Q(k) = A(k) Z_w(k) + B(k) conj Z_w(M'-k),
//   A(k) = [E - sin(th) w^k O] / M',  B(k) = i cos(th) w^k O / M',
// th = 2 pi k / M, E/O the split of C (so C(k) = E + w^k O,
// C(k+M') = E - w^k O); the 1/M' of the inverse transform is folded in.
template <int EPT, int NT = 256>
__global__ __launch_bounds__(NT) void k_pass2_embed(ConvGeom g, const float2* __restrict__ T1,
                                                     float4* __restrict__ AB) {
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int M1 = g.M1, M2 = g.M2;
    float2* buf = smem;
    float2* tw = smem + 2 * M2;
    const RowPair rp(blockIdx.x, M1, M2);
    for (int t = tid; t < M2; t += nthr) tw[t] = g.tw2[t];
    load_rows<EPT>(buf, T1, rp, M2, tid, nthr);
    lds_barrier();
    lds_fft<-1, EPT>(buf, g.st2, rp.nseq, M2, tw, tid, nthr);
    const double invMp = 1.0 / (double)g.Mp;
    for (int idx = tid; idx < rp.nseq * M2; idx += nthr) {
        const int s = idx / M2, e = idx - s * M2;
        const int k1 = rp.row(s);
        int pk1, pk2;
        if (k1 == 0) {
            pk1 = 0;
            pk2 = (M2 - e) % M2;
        } else {
            pk1 = M1 - k1;
            pk2 = M2 - 1 - e;
        }
        const int ps = (pk1 == rp.a) ? 0 : 1;
        const float2 z = buf[s * M2 + e], zp = buf[ps * M2 + pk2];
        const SplitD d = split_eo(z, zp);
        const long long k = (long long)k1 + (long long)M1 * e;
        double sn, cs;
        sincospi(2.0 * (double)k / (double)g.M, &sn, &cs);
        // w^k = cs - i sn ; w^k O
        const double wor = cs * d.orr + sn * d.oi;
        const double woi = cs * d.oi - sn * d.orr;
        const double ar = (d.er - sn * wor) * invMp, ai = (d.ei - sn * woi) * invMp;
        // B = i cs (w^k O) / M'
        const double br = -cs * woi * invMp, bi = cs * wor * invMp;
        AB[(long long)k1 * M2 + e] = make_float4((float)ar, (float)ai, (float)br, (float)bi);
    }
}

// Rank-1 Hankelization of each group (Algorithm 4, summed over the group's
// triples before the single inverse transform):
//   G(k) += sigma_i U_i(k) V_i(k),  G(k+M') += sigma_i U_i(k+M') V_i(k+M'),
// then Q(k) = [(G(k) + G(k+M'))/2 + i (G(k) - G(k+M')) / (2 w^k)] / M'.
// NP = bin pairs per thread (M2 <= kReconThreads * NP): the FP64 accumulators of NP
// pairs live in registers, so NP is the smallest that covers the row (1 for rows of up
// to 1024 points) rather than the largest (4 would spill them to scratch memory).
constexpr int kReconThreads = 1024;
template <int EPT, int NP, typename F2 = FftGeneric>
__global__ __launch_bounds__(kReconThreads) void k_pass2_recon(ConvGeom g, const float2* __restrict__ T1all,
                                                              int k, const double* __restrict__ sigma,
                                                              const int* __restrict__ offs,
                                                              const int* __restrict__ members, int g0,
                                                              float2* __restrict__ T2all) {
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int M1 = g.M1, M2 = g.M2;
    const long long Mp = g.Mp;
    float2* buf = smem;
    float2* tw = smem + 2 * M2;
    const RowPair rp(blockIdx.x, M1, M2);
    const int grp = g0 + blockIdx.y;
    for (int t = tid; t < M2; t += nthr) tw[t] = g.tw2[t];

    float2 zu0[NP], zu1[NP];
    double g00r[NP], g00i[NP], g01r[NP], g01i[NP];
    double g10r[NP], g10i[NP], g11r[NP], g11i[NP];
    double w0r[NP], w0i[NP], w1r[NP], w1i[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        g00r[i] = g00i[i] = g01r[i] = g01i[i] = g10r[i] = g10i[i] = g11r[i] = g11i[i] = 0.0;
        const int p = tid + i * nthr;
        w0r[i] = w0i[i] = w1r[i] = w1i[i] = 0.0;
        if (p < rp.npairs) {
            int s0, e0, s1, e1;
            rp.pair(p, M2, s0, e0, s1, e1);
            const long long ka = (long long)rp.row(s0) + (long long)M1 * e0;
            const long long kb = (long long)rp.row(s1) + (long long)M1 * e1;
            double sn, cs;
            sincospi(2.0 * (double)ka / (double)g.M, &sn, &cs);
            w0r[i] = cs;
            w0i[i] = -sn;
            sincospi(2.0 * (double)kb / (double)g.M, &sn, &cs);
            w1r[i] = cs;
            w1i[i] = -sn;
        }
    }
    const int mb = offs[grp], me = offs[grp + 1];
    for (int mi = mb; mi < me; ++mi) {
        const int tri = members[mi];
        const double sg = sigma[tri];
        // u_i spectrum rows
        lds_barrier();
        load_rows<EPT>(buf, T1all + (long long)tri * Mp, rp, M2, tid, nthr);
        lds_barrier();
        fft_run_waves<-1, EPT>(F2{}, buf, g.st2, rp.nseq, M2, tw, tid, nthr);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = tid + i * nthr;
            if (p < rp.npairs) {
                int s0, e0, s1, e1;
                rp.pair(p, M2, s0, e0, s1, e1);
                zu0[i] = buf[s0 * M2 + e0];
                zu1[i] = buf[s1 * M2 + e1];
            }
        }
        lds_barrier();
        // v_i spectrum rows
        load_rows<EPT>(buf, T1all + (long long)(k + tri) * Mp, rp, M2, tid, nthr);
        lds_barrier();
        fft_run_waves<-1, EPT>(F2{}, buf, g.st2, rp.nseq, M2, tw, tid, nthr);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = tid + i * nthr;
            if (p < rp.npairs) {
                int s0, e0, s1, e1;
                rp.pair(p, M2, s0, e0, s1, e1);
                const float2 zv0 = buf[s0 * M2 + e0], zv1 = buf[s1 * M2 + e1];
                // element 0 (bin ka) and element 1 (bin kb = M'-ka)
                for (int side = 0; side < 2; ++side) {
                    const SplitD su = side == 0 ? split_eo(zu0[i], zu1[i]) : split_eo(zu1[i], zu0[i]);
                    const SplitD sv = side == 0 ? split_eo(zv0, zv1) : split_eo(zv1, zv0);
                    const double wr = side == 0 ? w0r[i] : w1r[i], wi = side == 0 ? w0i[i] : w1i[i];
                    // U(k) = E + w O ; U(k+M') = E - w O
                    const double uor = wr * su.orr - wi * su.oi, uoi = wr * su.oi + wi * su.orr;
                    const double vor = wr * sv.orr - wi * sv.oi, voi = wr * sv.oi + wi * sv.orr;
                    const double ua_r = su.er + uor, ua_i = su.ei + uoi, ub_r = su.er - uor, ub_i = su.ei - uoi;
                    const double va_r = sv.er + vor, va_i = sv.ei + voi, vb_r = sv.er - vor, vb_i = sv.ei - voi;
                    const double pa_r = ua_r * va_r - ua_i * va_i, pa_i = ua_r * va_i + ua_i * va_r;
                    const double pb_r = ub_r * vb_r - ub_i * vb_i, pb_i = ub_r * vb_i + ub_i * vb_r;
                    if (side == 0) {
                        g00r[i] += sg * pa_r; g00i[i] += sg * pa_i;
                        g01r[i] += sg * pb_r; g01i[i] += sg * pb_i;
                    } else {
                        g10r[i] += sg * pa_r; g10i[i] += sg * pa_i;
                        g11r[i] += sg * pb_r; g11i[i] += sg * pb_i;
                    }
                }
            }
        }
    }
    lds_barrier();
    const double invMp = 1.0 / (double)Mp;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * nthr;
        if (p < rp.npairs) {
            int s0, e0, s1, e1;
            rp.pair(p, M2, s0, e0, s1, e1);
            for (int side = 0; side < 2; ++side) {
                const double ga_r = side == 0 ? g00r[i] : g10r[i], ga_i = side == 0 ? g00i[i] : g10i[i];
                const double gb_r = side == 0 ? g01r[i] : g11r[i], gb_i = side == 0 ? g01i[i] : g11i[i];
                const double wr = side == 0 ? w0r[i] : w1r[i], wi = side == 0 ? w0i[i] : w1i[i];
                // (G(k) - G(k+M')) / w^k = (dr + i di) * conj(w)   (|w| = 1)
                const double dr = ga_r - gb_r, di = ga_i - gb_i;
                const double tr = dr * wr + di * wi, ti = di * wr - dr * wi;
                // Q = (ga + gb)/2 + i t/2
                const double qr = 0.5 * (ga_r + gb_r) - 0.5 * ti;
                const double qi = 0.5 * (ga_i + gb_i) + 0.5 * tr;
                const float2 q = make_float2((float)(qr * invMp), (float)(qi * invMp));
                if (side == 0) buf[s0 * M2 + e0] = q;
                else if (s0 != s1 || e0 != e1) buf[s1 * M2 + e1] = q;
            }
        }
    }
    lds_barrier();
    fft_run_waves<1, EPT>(F2{}, buf, g.st2, rp.nseq, M2, tw, tid, nthr);
    store_rows<EPT>(buf, T2all + (long long)blockIdx.y * Mp, rp, M2, tid, nthr);
}

// ---------------------------------------------------------------------------
// pass 3: conj twiddle, inverse column FFTs, emit y[2n], y[2n+1]

// antidiagonal length of position n of a length-n_all series with window L
__device__ __forceinline__ long long count1(long long n, long long n_all, long long L, long long K) {
    long long c = n + 1;
    if (L < c) c = L;
    if (K < c) c = K;
    if (n_all - n < c) c = n_all - n;
    return c;
}

template <int MODE>
__device__ __forceinline__ void p3_emit(const P3Out& o, long long m, float val, float coef, int y) {
    if constexpr (MODE == OUT_SLICE) {
        long long t = m - (o.n_in - 1);
        if (t >= 0 && t < o.n_out) {
            if (o.pitch) {
                t = compress_index(t, o.pitch, o.wout);
                if (t < 0) return;
            }
            float r = val;
            if (o.prev) r -= coef * o.prev[t];
            o.out[t] = r;
        }
    } else {
        if (m < o.N) {
            long long c;
            if (o.pitch) {
                const long long i = m / o.pitch, j = m - i * o.pitch;
                c = count1(i, o.Nx, o.Lx, o.Kx) * count1(j, o.pitch, o.L, o.K);
            } else {
                c = count1(m, o.N, o.L, o.K);
            }
            o.out[(long long)y * o.ldo + m] = val / (float)c;
        }
    }
}

template <int MODE, int EPT, int NT = 256, typename F1 = FftGeneric, bool QTW = false>
__global__ __launch_bounds__(NT) void k_pass3(ConvGeom g, const float2* __restrict__ T2, P3Out o) {
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int CB = g.CB, M1 = g.M1, M2 = g.M2, ss = M1 + 1;
    float2* buf = smem;
    float2* tw = smem + CB * ss;
    const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
    const int y = blockIdx.y;
    const float2* in = T2 + (long long)y * g.Mp;
    // the first four elements per thread (with their twiddles) and the first pass twiddle
    // are loaded, at clamped positions, before any LDS write
    const int nz = CB * M1;
    float2 zv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = min(tid + i * nthr, nz - 1);
        const int c = idx % CB, k1 = idx / CB, n2 = min(c0 + c, M2 - 1);
        zv[i] = cmul(in[(long long)k1 * M2 + n2], cconj(twiddle_mp(g, (long long)n2 * k1)));
    }
    const int ntw = QTW ? M1 / 4 : M1;  // entries of the twiddle table
    const float2 tw0 = g.tw1[min(tid, ntw - 1)];
    if (tid < ntw) tw[tid] = tw0;
    for (int t = tid + nthr; t < ntw; t += nthr) tw[t] = g.tw1[t];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = tid + i * nthr;
        if (idx < nz) buf[(idx % CB) * ss + idx / CB] = c0 + idx % CB < M2 ? zv[i] : make_float2(0.0f, 0.0f);
    }
    for (int idx = tid + 4 * nthr; idx < nz; idx += nthr) {
        const int c = idx % CB, k1 = idx / CB, n2 = c0 + c;
        float2 z = make_float2(0.0f, 0.0f);
        if (n2 < M2) z = cmul(in[(long long)k1 * M2 + n2], cconj(twiddle_mp(g, (long long)n2 * k1)));
        buf[c * ss + k1] = z;
    }
    lds_barrier();
    if constexpr (QTW)
        fft_run_quarter<1, EPT>(F1{}, buf, CB, ss, tw, tid, nthr);
    else
        fft_run_waves<1, EPT>(F1{}, buf, g.st1, CB, ss, tw, tid, nthr);
    float coef = 0.0f;
    if constexpr (MODE == OUT_SLICE) {
        if (o.coef) coef = (float)(*o.coef);
    }
    for (int idx = tid; idx < CB * M1; idx += nthr) {
        const int c = idx % CB, n1 = idx / CB, n2 = c0 + c;
        if (n2 < M2) {
            const float2 q = buf[c * ss + n1];
            const long long n = (long long)M2 * n1 + n2;
            p3_emit<MODE>(o, 2 * n, q.x, coef, y);
            p3_emit<MODE>(o, 2 * n + 1, q.y, coef, y);
        }
    }
}

// ---------------------------------------------------------------------------
// Short antidiagonals of the grouped Hankelization, from the definition.
// The FP32 FFT leaves an absolute error of order eps * sigma |u| |v| on every
// convolution entry; averaging divides it by the antidiagonal length cnt[n],
// so near the two ends of the series (cnt ~ 1) the FFT value is recomputed
// directly: g[n] = sum_i sigma_i sum_{a+b=n} u_i[a] v_i[b] / cnt[n]
// (FP64 sums of exact FP32 products) for every n with cnt[n] <= kEdgeCnt.

__global__ __launch_bounds__(256) void k_recon_edges(const double* __restrict__ sigma, const float* __restrict__ U,
                                                     long long ldu, const float* __restrict__ V, long long ldv,
                                                     const int* __restrict__ offs, const int* __restrict__ members,
                                                     long long N, long long L, long long K, float* __restrict__ out,
                                                     long long ldo) {
    const int grp = blockIdx.y;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long lmin = L < K ? L : K;
    const long long ne = lmin <= kEdgeCnt ? N : 2LL * kEdgeCnt;
    if (idx >= ne) return;
    const long long n = (lmin <= kEdgeCnt || idx < kEdgeCnt) ? idx : N - 2LL * kEdgeCnt + idx;
    const long long a0 = n - K + 1 > 0 ? n - K + 1 : 0;
    const long long a1 = n < L - 1 ? n : L - 1;
    double acc = 0.0;
    for (int mi = offs[grp]; mi < offs[grp + 1]; ++mi) {
        const int i = members[mi];
        const float* u = U + (long long)i * ldu;
        const float* v = V + (long long)i * ldv;
        double s = 0.0;
        for (long long a = a0; a <= a1; ++a) s += (double)u[a] * (double)v[n - a];
        acc += sigma[i] * s;
    }
    out[(long long)grp * ldo + n] = (float)(acc / (double)(a1 - a0 + 1));
}

// The same sums for long series (min(L, K) > kEdgeCnt: the 2 kEdgeCnt positions of the
// two ends), a tile of kEdgeTile positions per workgroup: the stretch of u_i and v_i the
// tile needs is staged in LDS once per member, and kEdgeSlices threads share each
// position's sum over a (a = a0 + slice, a0 + slice + kEdgeSlices, ...), meeting in a
// fixed order at the end.
constexpr int kEdgeTile = 16;
constexpr int kEdgeSlices = 16;  // kEdgeTile * kEdgeSlices = 256 threads
__global__ __launch_bounds__(256) void k_recon_edges_tiled(const double* __restrict__ sigma,
                                                           const float* __restrict__ U, long long ldu,
                                                           const float* __restrict__ V, long long ldv,
                                                           const int* __restrict__ offs,
                                                           const int* __restrict__ members, long long N,
                                                           long long L, long long K, float* __restrict__ out,
                                                           long long ldo) {
    __shared__ float us[kEdgeCnt + kEdgeTile];
    __shared__ float vs[kEdgeCnt + kEdgeTile];
    __shared__ double red[kEdgeSlices][kEdgeTile];
    const int grp = blockIdx.y, tid = threadIdx.x;
    const int nl = tid % kEdgeTile, sl = tid / kEdgeTile;
    const long long idx0 = (long long)blockIdx.x * kEdgeTile;  // tiles never straddle the two ends
    const long long n0 = idx0 < kEdgeCnt ? idx0 : N - 2LL * kEdgeCnt + idx0;
    const long long n = n0 + nl;
    // the stretch of u and v the tile's positions read
    const long long amin = n0 - K + 1 > 0 ? n0 - K + 1 : 0;
    const long long amax = n0 + kEdgeTile - 1 < L - 1 ? n0 + kEdgeTile - 1 : L - 1;
    const long long bmin = n0 - amax > 0 ? n0 - amax : 0;
    const long long bmax = n0 + kEdgeTile - 1 - amin < K - 1 ? n0 + kEdgeTile - 1 - amin : K - 1;
    const long long a0 = n - K + 1 > 0 ? n - K + 1 : 0;
    const long long a1 = n < L - 1 ? n : L - 1;
    double acc = 0.0;
    for (int mi = offs[grp]; mi < offs[grp + 1]; ++mi) {
        const int i = members[mi];
        const float* u = U + (long long)i * ldu;
        const float* v = V + (long long)i * ldv;
        __syncthreads();  // the previous member's reads are done
        for (long long a = amin + tid; a <= amax; a += 256) us[a - amin] = u[a];
        for (long long b = bmin + tid; b <= bmax; b += 256) vs[b - bmin] = v[b];
        __syncthreads();
        double sum = 0.0;
        for (long long a = a0 + sl; a <= a1; a += kEdgeSlices) sum += (double)us[a - amin] * (double)vs[n - a - bmin];
        acc += sigma[i] * sum;
    }
    red[sl][nl] = acc;
    __syncthreads();
    if (sl == 0) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < kEdgeSlices; ++q) tot += red[q][nl];
        out[(long long)grp * ldo + n] = (float)(tot / (double)(a1 - a0 + 1));
    }
}

// The same for a 2D array (Nx x Ny, window Lx x Ly, U and V compressed row by
// row): every position whose count cnt_x(i) cnt_y(j) is at most kEdgeCnt is
// recomputed as sum_i sigma_i sum_{a+c=i, b+d=j} U_i[a, b] V_i[c, d] / count.
__global__ __launch_bounds__(256) void k_recon_edges_2d(const double* __restrict__ sigma, const float* __restrict__ U,
                                                        long long ldu, const float* __restrict__ V, long long ldv,
                                                        const int* __restrict__ offs, const int* __restrict__ members,
                                                        long long Nx, long long Ny, long long Lx, long long Ly,
                                                        float* __restrict__ out, long long ldo) {
    const int grp = blockIdx.y;
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Nx * Ny) return;
    const long long Kx = Nx - Lx + 1, Ky = Ny - Ly + 1;
    const long long i = m / Ny, j = m - i * Ny;
    const long long a0 = i - Kx + 1 > 0 ? i - Kx + 1 : 0, a1 = i < Lx - 1 ? i : Lx - 1;
    const long long b0 = j - Ky + 1 > 0 ? j - Ky + 1 : 0, b1 = j < Ly - 1 ? j : Ly - 1;
    const long long cnt = (a1 - a0 + 1) * (b1 - b0 + 1);
    if (cnt > kEdgeCnt) return;
    double acc = 0.0;
    for (int mi = offs[grp]; mi < offs[grp + 1]; ++mi) {
        const int q = members[mi];
        const float* u = U + (long long)q * ldu;
        const float* v = V + (long long)q * ldv;
        double s = 0.0;
        for (long long a = a0; a <= a1; ++a)
            for (long long b = b0; b <= b1; ++b) s += (double)u[a * Ly + b] * (double)v[(i - a) * Ky + (j - b)];
        acc += sigma[q] * s;
    }
    out[(long long)grp * ldo + m] = (float)(acc / (double)cnt);
}

// ---------------------------------------------------------------------------
// misc

__global__ void k_check_finite(const double* __restrict__ f, long long N, double* flag) {
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < N;
         t += (long long)gridDim.x * blockDim.x) {
        if (!isfinite(f[t])) *flag = 1.0;
    }
}

__global__ void k_fill_zero(double* p, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

__global__ void k_start_vector(float* r, long long n, unsigned long long seed) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) r[t] = gauss(seed, 0, t);
}

// ---------------------------------------------------------------------------
// classical Gram-Schmidt


// block-wide sum (any block of up to 1024 threads), fixed order, valid in every thread
// r <- r - basis * h (h in LDS), one workgroup
__device__ void blk_subtract(float* r, long long n, const float* basis, long long ld, int ncols,
                             const double* h) {
    for (long long t = threadIdx.x; t < n; t += blockDim.x) {
        double acc = r[t];
        for (int c = 0; c < ncols; ++c) acc -= (double)basis[(long long)c * ld + t] * h[c];
        r[t] = (float)acc;
    }
    __syncthreads();
}

// h[c] = <basis_c, r> for c < ncols, returns |r|^2, one workgroup
__device__ double blk_project(const float* r, long long n, const float* basis, long long ld, int ncols,
                              double* h, double* sh) {
    for (int c = 0; c < ncols; ++c) {
        double acc = 0.0;
        const float* col = basis + (long long)c * ld;
        for (long long t = threadIdx.x; t < n; t += blockDim.x) acc += (double)col[t] * (double)r[t];
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) h[c] = s;
    }
    double acc = 0.0;
    for (long long t = threadIdx.x; t < n; t += blockDim.x) acc += (double)r[t] * (double)r[t];
    const double rr = block_sum(acc, sh);
    __syncthreads();
    return rr;
}

// Coefficients h, the new B entry and the normalization (one workgroup).
//   common case: |r_new|^2 = |r|^2 - |h|^2 >= |r|^2 / 2  (one CGS pass suffices);
//   DGKS case  : a second projection is computed here and h replaced by it
//                after subtracting the first (r is updated in place);
//   breakdown  : the new vector is numerically in the span of the basis; the
//                B entry becomes 0 and a seeded random direction, made
//                orthogonal to the basis by two passes, continues the
//                recurrence.
//
// hs[0..ncols] holds the column sums on entry (hs[ncols] = |r|^2); bnorm is state[0].
__device__ void cgs_finish(const ReduceArgs& a, double* hs, double* sh, int& decision, double bnorm) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const double hh = sumsq_allwave(hs, a.ncols);  // as the pass-1 launches that fold this step
    const double rr = hs[a.ncols];
    double coef, scale;
    if (a.full) {
        for (int c = tid; c < a.ncols; c += nt) hs[c] = 0.0;
        coef = 0.0;
        scale = 0.0;
        if (a.dgks_flag && tid == 0) *a.dgks_flag = 0;
    } else {
        double a2 = rr - hh;
        const double thr = a.tol_bd * bnorm;
        if (tid == 0) decision = (a2 >= 0.5 * rr && sqrt(a2) > thr) ? 0 : 1;
        __syncthreads();
        if (decision == 0) {
            coef = sqrt(a2);
            scale = 1.0 / coef;
            if (a.dgks_flag && tid == 0) *a.dgks_flag = 0;
        } else if (a.dgks_flag) {
            // long vectors: the update writes r - basis h unscaled and the second pass runs
            // over the whole grid (the gated launches that follow); h stays in a.h
            if (tid == 0) {
                *a.dgks_flag = 1;
                *a.scale_out = 1.0;
                a.state[2] += 1.0;
            }
            return;
        } else {
            // second Gram-Schmidt pass on the updated vector
            blk_subtract(a.r, a.n, a.basis, a.ld, a.ncols, hs);
            __syncthreads();
            const double rr2 = blk_project(a.r, a.n, a.basis, a.ld, a.ncols, hs, sh);
            __syncthreads();
            double hh2 = 0.0;
            for (int c = tid; c < a.ncols; c += nt) hh2 += hs[c] * hs[c];
            hh2 = block_sum(hh2, sh);
            a2 = rr2 - hh2;
            if (tid == 0) decision = (a2 > 0.0 && sqrt(a2) > thr) ? 2 : 3;
            __syncthreads();
            if (decision == 2) {
                coef = sqrt(a2);
                scale = 1.0 / coef;
                if (tid == 0) a.state[2] += 1.0;
            } else {
                // breakdown: fresh direction
                coef = 0.0;
                const unsigned long long ctr = a.stream_ctr;
                for (long long t = tid; t < a.n; t += nt) {
                    if (a.segmented) {
                        const long long i = seg_natural(a.seg, t / a.seg.S, t % a.seg.S);
                        a.r[t] = i >= 0 ? gauss(a.seed, ctr, i) : 0.0f;
                    } else {
                        a.r[t] = gauss(a.seed, ctr, t);
                    }
                }
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    blk_project(a.r, a.n, a.basis, a.ld, a.ncols_bd, hs, sh);
                    __syncthreads();
                    blk_subtract(a.r, a.n, a.basis, a.ld, a.ncols_bd, hs);
                }
                const double rr3 = blk_project(a.r, a.n, a.basis, 0, 0, hs, sh);
                for (int c = tid; c < a.ncols_bd; c += nt) hs[c] = 0.0;
                scale = rr3 > 0.0 ? 1.0 / sqrt(rr3) : 0.0;
                if (tid == 0) a.state[1] += 1.0;
            }
        }
    }
    __syncthreads();
    for (int c = tid; c < a.ncols; c += nt) a.h[c] = hs[c];
    if (tid == 0) {
        *a.coef_out = coef;
        *a.scale_out = scale;
        if (a.track && coef > a.state[0]) a.state[0] = coef;
    }
}

// Projection h = basis^T r and |r|^2, FP64 sums of exact FP32 products, in
// (row chunk, column group of CJ columns) tiles: part[c * pstride + chunk] for
// c < ncols, and part[ncols * pstride + chunk] = the chunk's |r|^2 (column
// group 0).  A chunk is a.chunk_rows rows, summed in steps of kProjRows (one
// float4 row per thread) before the workgroup's reduction.
template <int CJ>
__global__ __launch_bounds__(256) void k_cgs_project(ReduceArgs a) {
    if (a.gate && *a.gate == 0) return;
    __shared__ double red[CJ + 1][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = blockIdx.y * CJ;
    const int nc = min(CJ, a.ncols - c0);
    const long long tend = min(a.n, (long long)(blockIdx.x + 1) * a.chunk_rows);
    double acc[CJ + 1];
#pragma unroll
    for (int c = 0; c <= CJ; ++c) acc[c] = 0.0;
    for (long long t = (long long)blockIdx.x * a.chunk_rows + 4 * tid; t < tend; t += kProjRows) {
        const float4 rv = rows4(a.r, t, a.n);
#pragma unroll
        for (int c = 0; c < CJ; ++c)
            if (c < nc) acc[c] += dot4(rows4(a.basis + (long long)(c0 + c) * a.ld, t, a.n), rv);
        if (blockIdx.y == 0) acc[CJ] += dot4(rv, rv);
    }
#pragma unroll
    for (int c = 0; c <= CJ; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[c][wave] = v;
    }
    __syncthreads();
    if (tid <= CJ) {
        const int c = tid;
        const double sum = red[c][0] + red[c][1] + red[c][2] + red[c][3];
        if (c < nc) a.part[(long long)(c0 + c) * a.pstride + blockIdx.x] = sum;
        if (c == CJ && blockIdx.y == 0) a.part[(long long)a.ncols * a.pstride + blockIdx.x] = sum;
    }
}

// Column sums for long vectors (many chunks): workgroup c adds part[c][chunk]
// over all chunks (thread-strided, then the block sum: a fixed order) into h[c].
__global__ __launch_bounds__(256) void k_cgs_colsum(ReduceArgs a) {
    if (a.gate && *a.gate == 0) return;
    __shared__ double sh[16];
    const double* row = a.part + (long long)blockIdx.x * a.pstride;
    double sum = 0.0;
    for (int ch = threadIdx.x; ch < a.nchunks; ch += 256) sum += row[ch];
    sum = block_sum(sum, sh);
    if (threadIdx.x == 0) a.h[blockIdx.x] = sum;
}

// One workgroup (1024 threads): h[c] = sum over chunks of part[c][chunk] (16
// lanes per column with their loads in flight together, then a fixed-order
// shuffle tree), kept in LDS for cgs_finish and written out; or the sums that
// k_cgs_colsum has already formed.
constexpr int kReduceThreads = 1024;
constexpr int kReduceLanes = 16;
__global__ __launch_bounds__(kReduceThreads) void k_cgs_reduce(ReduceArgs a) {
    if (a.gate && *a.gate == 0) return;
    // the early-exit flag is tested once the partial sums are loaded; a stopped launch
    // writes nothing
    const double stopv = a.stop ? *a.stop : 0.0;
    __shared__ double hs[kMaxCols + 1];
    __shared__ double sh[16];
    __shared__ int decision;
    const int tid = threadIdx.x;
    const double bnorm = a.state[0];
    if (!a.presummed) {
        const int l = tid % kReduceLanes;
        for (int c = tid / kReduceLanes; c <= a.ncols; c += kReduceThreads / kReduceLanes) {
            const double* row = a.part + (long long)c * a.pstride;
            double sum = 0.0;
#pragma unroll 16
            for (int ch = l; ch < a.nchunks; ch += kReduceLanes) sum += row[ch];
#pragma unroll
            for (int off = kReduceLanes / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, kReduceLanes);
            if (l == 0) {
                hs[c] = sum;
                if (stopv == 0.0) a.h[c] = sum;
            }
        }
    } else {
        for (int c = tid; c <= a.ncols; c += kReduceThreads) hs[c] = a.h[c];
    }
    if (stopv != 0.0) return;
    __syncthreads();
    cgs_finish(a, hs, sh, decision, bnorm);
    if (a.snap && threadIdx.x == 0) {  // thread 0 made every state update
        a.snap[0] = a.state[1];
        a.snap[1] = a.state[2];
    }
}

// out[t] = (r[t] - sum_c basis[c][t] h[c]) * scale, FP64 accumulation.  A
// workgroup covers 256 rows (4 per lane, float4); its 4 waves split the
// columns and their partial sums meet in LDS.
__global__ __launch_bounds__(256) void k_cgs_update(const float* r, const float* __restrict__ basis,
                                                    long long ld, int ncols, const double* __restrict__ h,
                                                    const double* __restrict__ scale, float* out,
                                                    long long n, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ double red[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long t = (long long)blockIdx.x * 256 + 4 * lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (t < n) {
#pragma unroll 4
        for (int c = wave; c < ncols; c += 4) {
            const float4 b = rows4(basis + (long long)c * ld, t, n);
            const double hc = h[c];
            a0 += (double)b.x * hc;
            a1 += (double)b.y * hc;
            a2 += (double)b.z * hc;
            a3 += (double)b.w * hc;
        }
    }
    red[wave][4 * lane + 0] = a0;
    red[wave][4 * lane + 1] = a1;
    red[wave][4 * lane + 2] = a2;
    red[wave][4 * lane + 3] = a3;
    __syncthreads();
    if (wave == 0 && t < n) {
        const double sc = *scale;
        const float4 rv = rows4(r, t, n);
        double s4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) s4[q] = red[0][4 * lane + q] + red[1][4 * lane + q] + red[2][4 * lane + q] + red[3][4 * lane + q];
        const float o0 = (float)(((double)rv.x - s4[0]) * sc), o1 = (float)(((double)rv.y - s4[1]) * sc);
        const float o2 = (float)(((double)rv.z - s4[2]) * sc), o3 = (float)(((double)rv.w - s4[3]) * sc);
        if (t + 3 < n) {
            *reinterpret_cast<float4*>(out + t) = make_float4(o0, o1, o2, o3);
        } else {
            out[t] = o0;
            if (t + 1 < n) out[t + 1] = o1;
            if (t + 2 < n) out[t + 2] = o2;
        }
    }
}

// ---------------------------------------------------------------------------
// Ritz vectors: out[i*ldo + t] = sum_c basis[c*ld + t] P[c*k + i]

// Short vectors: kRitzTile triples per workgroup with their coefficients staged in LDS.
constexpr int kRitzTile = 16;
__global__ __launch_bounds__(256) void k_ritz(const float* __restrict__ basis, long long ld, int ncols,
                                              const double* __restrict__ P, int k, float* __restrict__ out,
                                              long long ldo, long long n) {
    extern __shared__ double ps[];  // ncols x kRitzTile
    const int i0 = blockIdx.y * kRitzTile;
    const int kt = min(kRitzTile, k - i0);
    for (int idx = threadIdx.x; idx < ncols * kRitzTile; idx += 256) {
        const int c = idx / kRitzTile, i = idx - c * kRitzTile;
        ps[idx] = i < kt ? P[(long long)c * k + i0 + i] : 0.0;
    }
    __syncthreads();
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double acc[kRitzTile];
#pragma unroll
    for (int i = 0; i < kRitzTile; ++i) acc[i] = 0.0;
    for (int c = 0; c < ncols; ++c) {
        const double x = basis[(long long)c * ld + t];
#pragma unroll
        for (int i = 0; i < kRitzTile; ++i) acc[i] += x * ps[c * kRitzTile + i];
    }
#pragma unroll
    for (int i = 0; i < kRitzTile; ++i)
        if (i < kt) out[(long long)(i0 + i) * ldo + t] = (float)acc[i];
}

// Long vectors: one row per thread and kRitzWideTile triples per workgroup.  The
// coefficients of a column are the same for every lane, so they are read with a
// wave-uniform address (scalar loads, scalar operands of the FP64 FMAs) instead of
// LDS; fewer tiles also mean fewer passes over the basis.  Needs many waves per
// SIMD to hide the scalar-load latency of each column, hence long vectors only.
constexpr int kRitzWideTile = 32;
__global__ __launch_bounds__(256) void k_ritz_long(const float* __restrict__ basis, long long ld, int ncols,
                                              const double* __restrict__ P, int k, float* __restrict__ out,
                                              long long ldo, long long n) {
    const int i0 = blockIdx.y * kRitzWideTile;
    const int kt = min(kRitzWideTile, k - i0);
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double acc[kRitzWideTile];
#pragma unroll
    for (int i = 0; i < kRitzWideTile; ++i) acc[i] = 0.0;
    if (kt == kRitzWideTile) {
#pragma unroll 2
        for (int c = 0; c < ncols; ++c) {
            const double x = basis[(long long)c * ld + t];
            const double* pc = P + (long long)c * k + i0;
#pragma unroll
            for (int i = 0; i < kRitzWideTile; ++i) acc[i] += x * pc[i];
        }
    } else {
        for (int c = 0; c < ncols; ++c) {
            const double x = basis[(long long)c * ld + t];
            const double* pc = P + (long long)c * k + i0;
#pragma unroll
            for (int i = 0; i < kRitzWideTile; ++i)
                if (i < kt) acc[i] += x * pc[i];
        }
    }
#pragma unroll
    for (int i = 0; i < kRitzWideTile; ++i)
        if (i < kt) out[(long long)(i0 + i) * ldo + t] = (float)acc[i];
}

// ---------------------------------------------------------------------------
// launchers

static int ept_for(long long elems, int nthr) {
    const long long e = (elems + nthr - 1) / nthr;
    if (e <= 4) return 4;
    if (e <= 8) return 8;
    if (e <= 16) return 16;
    return 32;
}

// An FFT-pass workgroup holding more than 2048 points (up to 8192) runs
// kBigThreads threads with 8 points each (its own instantiation, NT =
// kBigThreads); smaller ones run 256 threads.
static bool pass_big(long long elems) { return elems > 2048; }

static size_t lds_p13(const ConvGeom& g) { return sizeof(float2) * ((size_t)g.CB * (g.M1 + 1) + g.M1); }
static size_t lds_p2(const ConvGeom& g) { return sizeof(float2) * (3 * (size_t)g.M2); }
// with quarter twiddle tables (the fixed-radix long-row kernels): under 80 KB, so that two
// workgroups share a CU
static size_t lds_p13q(const ConvGeom& g) { return sizeof(float2) * ((size_t)g.CB * (g.M1 + 1) + g.M1 / 4); }
static size_t lds_p2q(const ConvGeom& g) { return sizeof(float2) * (2 * (size_t)g.M2 + g.M2 / 4); }

#define SSA_EPT_SWITCH(ept, EXPR)             \
    switch (ept) {                            \
        case 4: { constexpr int E = 4; EXPR; } break;   \
        case 8: { constexpr int E = 8; EXPR; } break;   \
        case 16: { constexpr int E = 16; EXPR; } break; \
        default: { constexpr int E = 32; EXPR; } break; \
    }

hipError_t launch_tables(const ConvGeom& g, float2* tw1, float2* tw2, float2* tw_lo, float2* tw_hi,
                         hipStream_t s) {
    const long long S = 1LL << g.tw_shift;
    long long n = g.M1;
    if (g.M2 > n) n = g.M2;
    if (S > n) n = S;
    const long long nhi = (g.Mp + S - 1) / S;
    if (nhi > n) n = nhi;
    hipLaunchKernelGGL(k_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.M1, g.M2, g.Mp,
                       g.tw_shift, tw1, tw2, tw_lo, tw_hi);
    return hipGetLastError();
}

hipError_t launch_pass1(const ConvGeom& g, int mode, const P1In& in, int nvec, float2* T1, hipStream_t s) {
    const dim3 grid((g.M2 + g.CB - 1) / g.CB, nvec);
    const size_t lds = lds_p13(g);
    const long long elems = (long long)g.CB * g.M1;
    const int ept = ept_for(elems, 256);
    const dim3 big(kBigThreads);
    if (mode == IN_REV) {
        if (pass_big(elems) && FftPlanC::matches(g.st1))
            hipLaunchKernelGGL((k_pass1<IN_REV, 8, kBigThreads, FftPlanC, true>), grid, big, lds_p13q(g), s, g, in, T1);
        else if (pass_big(elems) && FftPlanD::matches(g.st1))
            hipLaunchKernelGGL((k_pass1<IN_REV, 8, kBigThreads, FftPlanD, true>), grid, big, lds_p13q(g), s, g, in, T1);
        else if (pass_big(elems))
            hipLaunchKernelGGL((k_pass1<IN_REV, 8, kBigThreads>), grid, big, lds, s, g, in, T1);
        else
            SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass1<IN_REV, E>), grid, dim3(256), lds, s, g, in, T1));
    } else if (mode == IN_SERIES) {
        if (pass_big(elems))
            hipLaunchKernelGGL((k_pass1<IN_SERIES, 8, kBigThreads>), grid, big, lds, s, g, in, T1);
        else
            SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass1<IN_SERIES, E>), grid, dim3(256), lds, s, g, in, T1));
    } else {
        if (pass_big(elems) && FftPlanC::matches(g.st1))
            hipLaunchKernelGGL((k_pass1<IN_VECS, 8, kBigThreads, FftPlanC, true>), grid, big, lds_p13q(g), s, g, in, T1);
        else if (pass_big(elems) && FftPlanD::matches(g.st1))
            hipLaunchKernelGGL((k_pass1<IN_VECS, 8, kBigThreads, FftPlanD, true>), grid, big, lds_p13q(g), s, g, in, T1);
        else if (pass_big(elems))
            hipLaunchKernelGGL((k_pass1<IN_VECS, 8, kBigThreads>), grid, big, lds, s, g, in, T1);
        else
            SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass1<IN_VECS, E>), grid, dim3(256), lds, s, g, in, T1));
    }
    return hipGetLastError();
}

hipError_t launch_pass2_matvec(const ConvGeom& g, const float4* AB, const float2* T1, float2* T2,
                               hipStream_t s) {
    const dim3 grid(g.M1 / 2 + 1);
    const int ept = ept_for(2LL * g.M2, 256);
    if (pass_big(2LL * g.M2) && FftPlanD::matches(g.st2))
        SSA_LAUNCH((k_pass2_matvec<8, kBigThreads, FftPlanD, true>), grid, dim3(kBigThreads), lds_p2q(g), s, g, AB, T1, T2);
    else if (pass_big(2LL * g.M2) && FftPlanC::matches(g.st2))
        SSA_LAUNCH((k_pass2_matvec<8, kBigThreads, FftPlanC, true>), grid, dim3(kBigThreads), lds_p2q(g), s, g, AB, T1, T2);
    else if (pass_big(2LL * g.M2))
        SSA_LAUNCH((k_pass2_matvec<8, kBigThreads>), grid, dim3(kBigThreads), lds_p2(g), s, g, AB, T1, T2);
    else if (ept == 4 && FftPlanB::matches(g.st2))
        SSA_LAUNCH((k_pass2_matvec<4, 256, FftPlanB>), grid, dim3(256), lds_p2(g), s, g, AB, T1, T2);
    else if (ept == 4 && FftPlanA::matches(g.st2))
        SSA_LAUNCH((k_pass2_matvec<4, 256, FftPlanA>), grid, dim3(256), lds_p2(g), s, g, AB, T1, T2);
    else
        SSA_EPT_SWITCH(ept, SSA_LAUNCH((k_pass2_matvec<E>), grid, dim3(256), lds_p2(g), s, g, AB, T1, T2));
    return hipGetLastError();
}

hipError_t launch_pass2_embed(const ConvGeom& g, const float2* T1, float4* AB, hipStream_t s) {
    const dim3 grid(g.M1 / 2 + 1);
    const int ept = ept_for(2LL * g.M2, 256);
    if (pass_big(2LL * g.M2))
        hipLaunchKernelGGL((k_pass2_embed<8, kBigThreads>), grid, dim3(kBigThreads), lds_p2(g), s, g, T1, AB);
    else
        SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass2_embed<E>), grid, dim3(256), lds_p2(g), s, g, T1, AB));
    return hipGetLastError();
}

hipError_t launch_pass2_recon(const ConvGeom& g, const float2* T1all, int k, const double* sigma,
                              const int* offs, const int* members, int g0, int ng, float2* T2all,
                              hipStream_t s) {
    const dim3 grid(g.M1 / 2 + 1, ng);
    const int ept = ept_for(2LL * g.M2, kReconThreads);
    const int np = (g.M2 + kReconThreads - 1) / kReconThreads;  // M2 <= 4096
#define SSA_RECON(NPV)                                                                                  \
    SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass2_recon<E, NPV>), grid, dim3(kReconThreads), lds_p2(g), s, g, \
                                           T1all, k, sigma, offs, members, g0, T2all))
    if (np <= 1 && ept == 4 && FftPlanB::matches(g.st2)) {
        hipLaunchKernelGGL((k_pass2_recon<4, 1, FftPlanB>), grid, dim3(kReconThreads), lds_p2(g), s, g, T1all, k,
                           sigma, offs, members, g0, T2all);
    } else if (np <= 1 && ept == 4 && FftPlanA::matches(g.st2)) {
        hipLaunchKernelGGL((k_pass2_recon<4, 1, FftPlanA>), grid, dim3(kReconThreads), lds_p2(g), s, g, T1all, k,
                           sigma, offs, members, g0, T2all);
    } else if (np == 4 && ept == 8 && FftPlanD::matches(g.st2)) {
        hipLaunchKernelGGL((k_pass2_recon<8, 4, FftPlanD>), grid, dim3(kReconThreads), lds_p2(g), s, g, T1all, k,
                           sigma, offs, members, g0, T2all);
    } else if (np == 2 && ept == 4 && FftPlanC::matches(g.st2)) {
        hipLaunchKernelGGL((k_pass2_recon<4, 2, FftPlanC>), grid, dim3(kReconThreads), lds_p2(g), s, g, T1all, k,
                           sigma, offs, members, g0, T2all);
    } else if (np <= 1) {
        SSA_RECON(1);
    } else if (np <= 2) {
        SSA_RECON(2);
    } else {
        SSA_RECON(4);
    }
#undef SSA_RECON
    return hipGetLastError();
}

hipError_t launch_pass3(const ConvGeom& g, int mode, const float2* T2, const P3Out& o, int nvec,
                        hipStream_t s) {
    const dim3 grid((g.M2 + g.CB - 1) / g.CB, nvec);
    const size_t lds = lds_p13(g);
    const long long elems = (long long)g.CB * g.M1;
    const int ept = ept_for(elems, 256);
    const dim3 big(kBigThreads);
    if (mode == OUT_SLICE) {
        if (pass_big(elems) && FftPlanC::matches(g.st1))
            hipLaunchKernelGGL((k_pass3<OUT_SLICE, 8, kBigThreads, FftPlanC, true>), grid, big, lds_p13q(g), s, g, T2, o);
        else if (pass_big(elems) && FftPlanD::matches(g.st1))
            hipLaunchKernelGGL((k_pass3<OUT_SLICE, 8, kBigThreads, FftPlanD, true>), grid, big, lds_p13q(g), s, g, T2, o);
        else if (pass_big(elems))
            hipLaunchKernelGGL((k_pass3<OUT_SLICE, 8, kBigThreads>), grid, big, lds, s, g, T2, o);
        else
            SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass3<OUT_SLICE, E>), grid, dim3(256), lds, s, g, T2, o));
    } else {
        if (pass_big(elems) && FftPlanC::matches(g.st1))
            hipLaunchKernelGGL((k_pass3<OUT_HANKEL, 8, kBigThreads, FftPlanC, true>), grid, big, lds_p13q(g), s, g, T2, o);
        else if (pass_big(elems) && FftPlanD::matches(g.st1))
            hipLaunchKernelGGL((k_pass3<OUT_HANKEL, 8, kBigThreads, FftPlanD, true>), grid, big, lds_p13q(g), s, g, T2, o);
        else if (pass_big(elems))
            hipLaunchKernelGGL((k_pass3<OUT_HANKEL, 8, kBigThreads>), grid, big, lds, s, g, T2, o);
        else
            SSA_EPT_SWITCH(ept, hipLaunchKernelGGL((k_pass3<OUT_HANKEL, E>), grid, dim3(256), lds, s, g, T2, o));
    }
    return hipGetLastError();
}

hipError_t launch_recon_edges_2d(const double* sigma, const float* U, long long ldu, const float* V,
                                 long long ldv, const int* offs, const int* members, int ng, long long Nx,
                                 long long Ny, long long Lx, long long Ly, float* out, long long ldo,
                                 hipStream_t s) {
    const long long n = Nx * Ny;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)ng);
    hipLaunchKernelGGL(k_recon_edges_2d, grid, dim3(256), 0, s, sigma, U, ldu, V, ldv, offs, members, Nx, Ny, Lx,
                       Ly, out, ldo);
    return hipGetLastError();
}

hipError_t launch_recon_edges(const double* sigma, const float* U, long long ldu, const float* V, long long ldv,
                              const int* offs, const int* members, int ng, long long N, long long L, long long K,
                              float* out, long long ldo, hipStream_t s) {
    const long long lmin = L < K ? L : K;
    if (lmin > kEdgeCnt) {
        static_assert(kEdgeCnt % kEdgeTile == 0, "edge tiles must not straddle the two ends");
        const dim3 grid((unsigned)(2 * kEdgeCnt / kEdgeTile), (unsigned)ng);
        hipLaunchKernelGGL(k_recon_edges_tiled, grid, dim3(256), 0, s, sigma, U, ldu, V, ldv, offs, members, N, L,
                           K, out, ldo);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((N + 255) / 256), (unsigned)ng);
    hipLaunchKernelGGL(k_recon_edges, grid, dim3(256), 0, s, sigma, U, ldu, V, ldv, offs, members, N, L, K, out, ldo);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* f, long long N, double* flag, hipStream_t s) {
    long long blocks = (N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, f, N, flag);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_start_vector(float* r, long long n, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(k_start_vector, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, n, seed);
    return hipGetLastError();
}

// Columns per projection workgroup: short vectors (few row chunks) are latency-bound and
// gain from more, smaller workgroups; long ones re-read r once per column group, so they
// take wider groups.
hipError_t launch_cgs_project(const ReduceArgs& a, hipStream_t s) {
    const unsigned nchunks = (unsigned)a.nchunks;
    const int cj = nchunks <= kProjNarrowChunks ? kProjColsNarrow : kProjCols;
    const unsigned ngrp = a.ncols > 0 ? (unsigned)((a.ncols + cj - 1) / cj) : 1u;
    if (cj == kProjColsNarrow)
        hipLaunchKernelGGL((k_cgs_project<kProjColsNarrow>), dim3(nchunks, ngrp), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_cgs_project<kProjCols>), dim3(nchunks, ngrp), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cgs_colsum(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_cgs_colsum, dim3((unsigned)(a.ncols + 1)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cgs_reduce(const ReduceArgs& a, hipStream_t s) {
    SSA_LAUNCH(k_cgs_reduce, dim3(1), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cgs_update(const float* r, const float* basis, long long ld, int ncols, const double* h,
                             const double* scale, float* out, long long n, const int* gate, hipStream_t s) {
    hipLaunchKernelGGL(k_cgs_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, basis, ld, ncols,
                       h, scale, out, n, gate);
    return hipGetLastError();
}

hipError_t launch_ritz(const float* basis, long long ld, int ncols, const double* P, int k, float* out,
                       long long ldo, long long n, hipStream_t s) {
    if (n >= kRitzWideRows) {
        const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((k + kRitzWideTile - 1) / kRitzWideTile));
        hipLaunchKernelGGL(k_ritz_long, grid, dim3(256), 0, s, basis, ld, ncols, P, k, out, ldo, n);
    } else {
        const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((k + kRitzTile - 1) / kRitzTile));
        const size_t lds = sizeof(double) * (size_t)ncols * kRitzTile;
        hipLaunchKernelGGL(k_ritz, grid, dim3(256), lds, s, basis, ld, ncols, P, k, out, ldo, n);
    }
    return hipGetLastError();
}

template <typename F>
static hipError_t allow_lds(F* f) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

hipError_t set_kernel_attributes() {
    hipError_t e = hipSuccess;
#define SSA_ALLOW(K)                              \
    do {                                          \
        hipError_t e2 = allow_lds(K);             \
        if (e2 != hipSuccess) e = e2;             \
    } while (0)
#define SSA_ALLOW_EPT(T)                          \
    SSA_ALLOW(T<4>); SSA_ALLOW(T<8>); SSA_ALLOW(T<16>); SSA_ALLOW(T<32>)
    SSA_ALLOW((k_pass1<IN_REV, 4>)); SSA_ALLOW((k_pass1<IN_REV, 8>)); SSA_ALLOW((k_pass1<IN_REV, 16>));
    SSA_ALLOW((k_pass1<IN_REV, 32>));
    SSA_ALLOW((k_pass1<IN_SERIES, 4>)); SSA_ALLOW((k_pass1<IN_SERIES, 8>)); SSA_ALLOW((k_pass1<IN_SERIES, 16>));
    SSA_ALLOW((k_pass1<IN_SERIES, 32>));
    SSA_ALLOW((k_pass1<IN_VECS, 4>)); SSA_ALLOW((k_pass1<IN_VECS, 8>)); SSA_ALLOW((k_pass1<IN_VECS, 16>));
    SSA_ALLOW((k_pass1<IN_VECS, 32>));
    SSA_ALLOW((k_pass3<OUT_SLICE, 4>)); SSA_ALLOW((k_pass3<OUT_SLICE, 8>)); SSA_ALLOW((k_pass3<OUT_SLICE, 16>));
    SSA_ALLOW((k_pass3<OUT_SLICE, 32>));
    SSA_ALLOW((k_pass3<OUT_HANKEL, 4>)); SSA_ALLOW((k_pass3<OUT_HANKEL, 8>));
    SSA_ALLOW((k_pass3<OUT_HANKEL, 16>)); SSA_ALLOW((k_pass3<OUT_HANKEL, 32>));
    SSA_ALLOW((k_pass1<IN_REV, 8, kBigThreads>)); SSA_ALLOW((k_pass1<IN_SERIES, 8, kBigThreads>));
    SSA_ALLOW((k_pass1<IN_VECS, 8, kBigThreads>));
    SSA_ALLOW((k_pass3<OUT_SLICE, 8, kBigThreads>)); SSA_ALLOW((k_pass3<OUT_HANKEL, 8, kBigThreads>));
    SSA_ALLOW((k_pass2_matvec<8, kBigThreads>)); SSA_ALLOW((k_pass2_embed<8, kBigThreads>));
    SSA_ALLOW((k_pass1<IN_REV, 8, kBigThreads, FftPlanC, true>));
    SSA_ALLOW((k_pass1<IN_REV, 8, kBigThreads, FftPlanD, true>));
    SSA_ALLOW((k_pass1<IN_VECS, 8, kBigThreads, FftPlanD, true>));
    SSA_ALLOW((k_pass3<OUT_SLICE, 8, kBigThreads, FftPlanD, true>));
    SSA_ALLOW((k_pass3<OUT_HANKEL, 8, kBigThreads, FftPlanD, true>));
    SSA_ALLOW((k_pass1<IN_VECS, 8, kBigThreads, FftPlanC, true>));
    SSA_ALLOW((k_pass3<OUT_SLICE, 8, kBigThreads, FftPlanC, true>));
    SSA_ALLOW((k_pass3<OUT_HANKEL, 8, kBigThreads, FftPlanC, true>));
    SSA_ALLOW((k_pass2_matvec<8, kBigThreads, FftPlanC, true>));
    SSA_ALLOW((k_pass2_matvec<8, kBigThreads, FftPlanD, true>));
    SSA_ALLOW_EPT(k_pass2_matvec);
    SSA_ALLOW((k_pass2_matvec<4, 256, FftPlanA>)); SSA_ALLOW((k_pass2_matvec<4, 256, FftPlanB>));
    SSA_ALLOW((k_pass2_recon<4, 1, FftPlanA>)); SSA_ALLOW((k_pass2_recon<4, 1, FftPlanB>));
    SSA_ALLOW((k_pass2_recon<8, 4, FftPlanD>)); SSA_ALLOW((k_pass2_recon<4, 2, FftPlanC>));
    SSA_ALLOW_EPT(k_pass2_embed);
#define SSA_ALLOW_RECON(NPV)                                                                   \
    SSA_ALLOW((k_pass2_recon<4, NPV>)); SSA_ALLOW((k_pass2_recon<8, NPV>));                      \
    SSA_ALLOW((k_pass2_recon<16, NPV>)); SSA_ALLOW((k_pass2_recon<32, NPV>))
    SSA_ALLOW_RECON(1);
    SSA_ALLOW_RECON(2);
    SSA_ALLOW_RECON(4);
#undef SSA_ALLOW_RECON
    SSA_ALLOW(k_ritz);
#undef SSA_ALLOW_EPT
#undef SSA_ALLOW
    return e;
}

}  // namespace ssa
