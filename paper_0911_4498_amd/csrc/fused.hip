// fused.hip -- the Lanczos half-step of the single-series path in three launches
// (four with the reduction as its own launch).
//
// Algorithm 1 alternates two half-steps; each is one trajectory-matrix product by
// FFT (Algorithms 2/3: pass 1 column FFTs, pass 2 row FFTs with the spectral
// operator, pass 3 inverse column FFTs) followed by classical Gram-Schmidt
// against the basis of its side (Sec. 3.2.2).  Kernel boundaries are the cheapest
// grid-wide synchronization on this GPU, so the work is cut where a grid-wide
// result is needed and fused everywhere else:
//
//   k_p1_update   the reduction of the previous half-step (every workgroup sums the
//                 partials itself: h, the new alpha or beta, the normalization; a
//                 DGKS pass or a breakdown sends the solve back to the four-launch
//                 form), then finishes that half-step's vector x = (r - B h) * scale
//                 (B its basis) and runs pass 1 of the product that takes x;
//   pass 2        unchanged (kernels.hip);
//   k_p3_project  pass 3, the three-term term r = y - coef * prev, and the
//                 projection partials <b_c, r> and |r|^2 of its block.
//
// In the four-launch form a single workgroup does the reduction in between
// (k_cgs_reduce, kernels.hip: DGKS, breakdown) and k_p1_update reads h and scale.
//
// The vectors of both bases live in the segment layout (SegLay): pass 3's
// workgroup owns a contiguous slot range of its output, and the reversed input of
// the next product maps each pass-1 column onto whole segments, so both fused
// kernels read the basis in coalesced float4 runs.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "ssa_internal.h"

namespace ssa {

// Threads of the fused kernels: 16 waves per workgroup keep enough basis loads in
// flight when one workgroup per CU streams its slice of the basis.
constexpr int kFusedThreads = 1024;
// basis columns a wave of k_p3_project handles at once (independent loads in flight)
constexpr int kProjUnroll = 4;
// pass-1 twiddles per thread in the preambles: M1 <= 4096
constexpr int kTwPer = 4;

// float2 words of the FFT buffer and its twiddles, rounded up to 16 bytes
__host__ __device__ inline int fused_fft_lds_words(const ConvGeom& g) {
    const int w = g.CB * (g.M1 + 1) + g.M1;
    return w + (w & 1);
}

// 32-bit forms of seg_lo / seg_count for these kernels: a fused plan holds at most 2^20
// rows, so every y index stays below 2^22, and a 32-bit division costs a fraction of the
// 64-bit one (these sit at the head of each workgroup's dependence chain).
__device__ __forceinline__ int seg_lo32(const SegLay& l, int n2, int e) {
    const int a = (int)l.o - 2 * n2 - e;
    const unsigned step = 2u * (unsigned)l.M2;
    return a <= 0 ? 0 : (int)(((unsigned)a + step - 1u) / step);
}

__device__ __forceinline__ int seg_count32(const SegLay& l, int n2, int e) {
    const int b = (int)(l.o + l.n) - 1 - 2 * n2 - e;
    if (b < 0) return 0;
    int hi = (int)((unsigned)b / (2u * (unsigned)l.M2));
    if (hi > l.M1 - 1) hi = l.M1 - 1;
    const int lo = seg_lo32(l, n2, e);
    return hi >= lo ? hi - lo + 1 : 0;
}

// Pass 3 + three-term term + projection partials.  Workgroup b (XCD-ordered)
// owns the columns [c0, c0 + CB) of the four-step layout, i.e. the output slots
// [2*c0*S, 2*(c0 + CB)*S).  The loads that do not depend on the transform (the
// three-term vector and the first basis columns of each wave) are issued before
// it, so their latency hides behind the column FFT.
template <int EPT, typename F1 = FftGeneric>
__global__ __launch_bounds__(kFusedThreads) void k_p3_project(ConvGeom g, const float2* __restrict__ T2, P3Seg a) {
    // the early-exit flag is read here and tested once the loads below are in flight
    const double stopv = g.stop ? *g.stop : 0.0;
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int kWaves = kFusedThreads / 64;
    const int CB = g.CB, M1 = g.M1, M2 = g.M2, ss = M1 + 1;
    const int S = a.lay.S;
    float2* buf = smem;             // CB x (M1 + 1)
    float2* tw = buf + CB * ss;     // M1
    float* rs = reinterpret_cast<float*>(smem + fused_fft_lds_words(g));  // 2 * CB * S floats
    const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
    const int ncb = min(CB, M2 - c0);  // columns of this block inside the transform
    const int nsl = 2 * ncb * S;
    const int nf = nsl / 4;
    const long long base = 2LL * c0 * S;
    const float cf = (a.prev && a.coef) ? (float)(*a.coef) : 0.0f;
    // (the loads below are unconditional at clamped, in-bounds positions: branches around
    // them would make the compiler wait for each one in turn)
    const float pv0 = a.prev ? a.prev[base + min(tid, nsl - 1)] : 0.0f;
    // (not in the 8-point instantiation for long rows: capped at 128 VGPRs, it would spill)
    constexpr int kPre = EPT >= 8 ? 0 : kProjUnroll;
    float4 pre[kPre > 0 ? kPre : 1];
#pragma unroll
    for (int u = 0; u < (kPre > 0 ? kPre : 1); ++u) pre[u] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const int c = wave * kProjUnroll + u;  // wave-uniform
        if (c < a.ncols) pre[u] = reinterpret_cast<const float4*>(a.basis + (long long)c * a.ld + base)[min(lane, nf - 1)];
    }
    // twiddles and the column elements (with their four-step twiddles) in batches of four
    // per thread, each batch's loads issued before its LDS writes (at clamped positions)
    // (a wave whose first index is past the data skips the load: a wave-uniform branch)
    const int wave0 = tid & ~63;
    float2 twv[kTwPer];
#pragma unroll
    for (int i = 0; i < kTwPer; ++i)
        if (wave0 + i * kFusedThreads < M1) twv[i] = g.tw1[min(tid + i * kFusedThreads, M1 - 1)];
    const int nz = CB * M1;  // <= EPT * kFusedThreads
#pragma unroll
    for (int b = 0; b < EPT; b += 4) {
        float2 zv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (wave0 + (b + i) * kFusedThreads >= nz) continue;
            const int idx = min(tid + (b + i) * kFusedThreads, nz - 1);
            const int c = idx % CB, k1 = idx / CB, n2 = min(c0 + c, M2 - 1);
            zv[i] = cmul(T2[(long long)k1 * M2 + n2], cconj(twiddle_mp(g, (long long)n2 * k1)));
        }
        if (b == 0) {
#pragma unroll
            for (int i = 0; i < kTwPer; ++i)
                if (tid + i * kFusedThreads < M1) tw[tid + i * kFusedThreads] = twv[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + (b + i) * kFusedThreads;
            if (idx < nz) {
                const int c = idx % CB, k1 = idx / CB;
                buf[c * ss + k1] = c0 + c < M2 ? zv[i] : make_float2(0.0f, 0.0f);
            }
        }
    }
    for (int idx = tid + EPT * kFusedThreads; idx < nz; idx += kFusedThreads) {  // (none when nz <= EPT * 1024)
        const int c = idx % CB, k1 = idx / CB, n2 = c0 + c;
        float2 z = make_float2(0.0f, 0.0f);
        if (n2 < M2) z = cmul(T2[(long long)k1 * M2 + n2], cconj(twiddle_mp(g, (long long)n2 * k1)));
        buf[c * ss + k1] = z;
    }
    if (stopv != 0.0) return;
    lds_barrier();
    fft_run_waves<1, EPT>(F1{}, buf, g.st1, CB, ss, tw, tid, kFusedThreads);
    for (int q = tid; q < nsl; q += kFusedThreads) {
        const int sg = q / S, t = q - sg * S;
        const int c = sg >> 1, e = sg & 1, n2 = c0 + c;
        float v = 0.0f;
        if (t < seg_count32(a.lay, n2, e)) {
            const float2 z = buf[c * ss + seg_lo32(a.lay, n2, e) + t];
            v = e ? z.y : z.x;
            if (a.prev) v -= cf * (q == tid ? pv0 : a.prev[base + q]);
        }
        rs[q] = v;
        a.r[base + q] = v;
    }
    lds_barrier();
    // partials: the waves split the columns (column ncols stands for |r|^2), the lanes
    // split the float4 groups of the block; FP64 sums of exact FP32 products
    const float4* r4 = reinterpret_cast<const float4*>(rs);
    const int ncol = a.ncols + 1;
    for (int cb0 = wave * kProjUnroll; cb0 < ncol; cb0 += kWaves * kProjUnroll) {
        const bool first = cb0 == wave * kProjUnroll;  // wave-uniform
        double acc[kProjUnroll];
#pragma unroll
        for (int u = 0; u < kProjUnroll; ++u) acc[u] = 0.0;
        for (int f = lane; f < nf; f += 64) {
            const float4 rv = r4[f];
            float4 bv[kProjUnroll];
            if (kPre > 0 && first && f == lane) {  // wave-uniform
#pragma unroll
                for (int u = 0; u < kProjUnroll; ++u) bv[u] = cb0 + u < a.ncols ? pre[u < kPre ? u : 0] : rv;
            } else {
                // all four loads in flight together: clamped (in-bounds) columns, then the
                // columns past the basis take r itself (its |r|^2)
                const int cmax = max(a.ncols - 1, 0);
#pragma unroll
                for (int u = 0; u < kProjUnroll; ++u)
                    bv[u] = reinterpret_cast<const float4*>(a.basis + (long long)min(cb0 + u, cmax) * a.ld + base)[f];
#pragma unroll
                for (int u = 0; u < kProjUnroll; ++u)
                    if (cb0 + u >= a.ncols) bv[u] = rv;
            }
#pragma unroll
            for (int u = 0; u < kProjUnroll; ++u) acc[u] += dot4(bv[u], rv);
        }
#pragma unroll
        for (int u = 0; u < kProjUnroll; ++u) {
            const double sum = wave_sum(acc[u]);
            const int c = cb0 + u;
            if (lane == 0 && c < ncol) a.part[(long long)c * a.pstride + blockIdx.x] = sum;
        }
    }
}

// Finishing the previous vector + pass 1 of the product that takes it.  The
// workgroup owns the columns [c0, c0 + CB) of pass 1; element (n1, n2, e) of the
// reversed input is natural element n_in - 1 - m (m = 2*(M2*n1 + n2) + e) of x,
// which sits at y index m' = N - 1 - m of x's layout: for fixed (n2, e) that is one
// segment s' whose slot t' holds n1 = Q - seg_lo(s') - t'.
struct SegSrc {
    long long pos;  // stored position of slot 0 of the source segment
    int lo, cnt, Q;  // its first n1', its element count (0: padding only), n1 = Q - n1'
};

// Source segment of local segment sl = 2 c + e (pass-1 column c0 + c, parity e).  A =
// m' - 2 M2 n1 for this (n2, e); over all pairs A runs through 2 M2 consecutive
// integers, so every segment of x is the source of exactly one pair.  A < 0 holds no
// element of x (m' < 0): its segment only gets its zeros written.
__device__ __forceinline__ SegSrc seg_source(const P1Seg& a, int M2, int S, int c0, int sl) {
    const int c = sl >> 1, e = sl & 1, n2 = c0 + c;
    const int A = (int)a.N - 1 - e - 2 * n2;  // N < 2^22 on the fused path
    const int ep = A & 1;
    const int H = (A - ep) / 2;  // exact
    int n2p, Q = 0;
    if (H >= 0) {
        Q = (int)((unsigned)H / (unsigned)M2);
        n2p = H - Q * M2;
    } else {
        n2p = ((H % M2) + M2) % M2;
    }
    SegSrc d;
    d.pos = (long long)(2 * n2p + ep) * S;
    d.Q = A >= 0 ? Q : 0;
    d.lo = seg_lo32(a.lay, n2p, ep);
    d.cnt = A >= 0 ? seg_count32(a.lay, n2p, ep) : 0;
    return d;
}

// Sum over the columns c = slice, slice + nslice, ... of basis[c][p..p+3] h[c] for
// float4 group f of the workgroup's source segments (nothing for a missing segment).
// The first kUpdPre columns may come preloaded (use_pre).
constexpr int kUpdPre = 4;
constexpr int kHPer = 2;   // h values per thread: ncols <= kMaxCols
static_assert(kHPer * kFusedThreads >= 1024 + 1, "h and |r|^2 fit the preamble loads (ncols <= d_max <= 1024)");
__device__ __forceinline__ void fused_accumulate(const P1Seg& a, const double* hs, const SegSrc* src, int gps, int f,
                                                 int slice, int nslice, double (&x)[4], const float4 (&pre)[kUpdPre],
                                                 bool use_pre) {
    x[0] = x[1] = x[2] = x[3] = 0.0;
    const int sg = f / gps;
    if (4 * (f - sg * gps) >= src[sg].cnt) return;  // padding slots only
    const long long p = src[sg].pos + 4LL * (f - sg * gps);
    int c = slice;
    if (use_pre) {
#pragma unroll
        for (int u = 0; u < kUpdPre; ++u, c += nslice) {
            if (c >= a.ncols) break;
            const double hc = hs[c];
            x[0] += (double)pre[u].x * hc;
            x[1] += (double)pre[u].y * hc;
            x[2] += (double)pre[u].z * hc;
            x[3] += (double)pre[u].w * hc;
        }
    }
    // four columns' loads in flight at a time (clamped columns, unconditional loads), added
    // in column order
    for (; c < a.ncols; c += 4 * nslice) {
        float4 b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            b[u] = *reinterpret_cast<const float4*>(a.basis + (long long)min(c + u * nslice, a.ncols - 1) * a.ld + p);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (c + u * nslice >= a.ncols) break;
            const double hc = hs[c + u * nslice];
            x[0] += (double)b[u].x * hc;
            x[1] += (double)b[u].y * hc;
            x[2] += (double)b[u].z * hc;
            x[3] += (double)b[u].w * hc;
        }
    }
}

// The four slots of r in float4 group f of the source segments (zeros past the segment's
// elements).
__device__ __forceinline__ float4 fused_load_r(const P1Seg& a, const SegSrc& d, int gps, int f, int sg) {
    const int tq0 = 4 * (f - sg * gps);
    return tq0 < d.cnt ? *reinterpret_cast<const float4*>(a.r + d.pos + tq0) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// x = (r - sum) * scale at the four slots of group f (rv: r there): written to the
// output column (zero in padding slots) and placed in the pass-1 buffer at its (n1, e).
__device__ __forceinline__ void fused_finish_group(const P1Seg& a, const SegSrc* src, int gps, int f,
                                                   const double (&x)[4], double scale, float2* buf, int ss,
                                                   float4 rv) {
    const int sg = f / gps;
    const SegSrc d = src[sg];
    const int tq0 = 4 * (f - sg * gps);
    const long long p = d.pos + tq0;
    const float r4[4] = {rv.x, rv.y, rv.z, rv.w};
    float o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int tq = tq0 + u;
        o[u] = 0.0f;
        if (tq < d.cnt) {
            o[u] = (float)(((double)r4[u] - x[u]) * scale);
            float2* z = &buf[(sg >> 1) * ss + (d.Q - d.lo - tq)];
            if (sg & 1) z->y = o[u];
            else z->x = o[u];
        }
    }
    *reinterpret_cast<float4*>(a.out + p) = make_float4(o[0], o[1], o[2], o[3]);
}

// The folded reduction, first part: hs[c] = sum over chunks of part[c][chunk] for c <=
// ncols, in the reduction kernel's order (16 lanes per column, each adding its chunks in
// sequence, then a shuffle tree).  The first 64 columns' loads (kFoldPer per lane) are
// issued at the head of the kernel (fold_load), so the sums run while the basis loads
// are in flight; further columns are loaded here.
constexpr int kFoldLanes = 16;
constexpr int kFoldPer = 16;  // chunks per lane: nchunks <= kFoldLanes * kFoldPer
static_assert(kFoldLanes * kFoldPer == kFoldMaxChunks, "fold lanes cover the partials");
__device__ __forceinline__ void fold_load(const FoldRed& f, int ncols, int tid, double (&pv)[kFoldPer]) {
    // unconditional loads at clamped (in-bounds) rows and chunks; fold_sums adds only the
    // valid ones
    const int l = tid % kFoldLanes, c = min(tid / kFoldLanes, ncols);
    if ((tid & ~63) / kFoldLanes > ncols) return;  // the wave's columns are all past ncols
    const double* row = f.part + (long long)c * f.pstride;
#pragma unroll
    for (int i = 0; i < kFoldPer; ++i)
        if (i * kFoldLanes < f.nchunks) pv[i] = row[min(l + i * kFoldLanes, f.nchunks - 1)];
}

__device__ __forceinline__ void fold_sums(const FoldRed& f, int ncols, double* hs, int tid,
                                          const double (&pv)[kFoldPer]) {
    const int l = tid % kFoldLanes;
    for (int c = tid / kFoldLanes; c <= ncols; c += kFusedThreads / kFoldLanes) {
        const double* row = f.part + (long long)c * f.pstride;
        double sum = 0.0;
        if (c < kFusedThreads / kFoldLanes) {
#pragma unroll
            for (int i = 0; i < kFoldPer; ++i)
                if (l + i * kFoldLanes < f.nchunks) sum += pv[i];
        } else {
#pragma unroll 16
            for (int ch = l; ch < f.nchunks; ch += kFoldLanes) sum += row[ch];
        }
#pragma unroll
        for (int off = kFoldLanes / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, kFoldLanes);
        if (l == 0) hs[c] = sum;
    }
}

// The same column sums as a launch of their own, for many columns (the pass-1 launch then
// reads ncols + 1 doubles): a wave sums four columns in fold_sums' order, so the bits are
// the same.  Each pass-1 workgroup would otherwise fetch all (ncols + 1) * nchunks partials
// through its own CU, whose outstanding misses bound the rate; spread over many workgroups
// each CU fetches a few columns.
__global__ __launch_bounds__(64) void k_fold_sums(FoldRed f, int ncols) {
    if (*f.fail != 0.0) return;  // the solve has stopped (the test's done flag)
    const int lane = threadIdx.x, l = lane % kFoldLanes;
    const int c = blockIdx.x * (64 / kFoldLanes) + lane / kFoldLanes;
    if (c > ncols) return;  // whole 16-lane groups
    const double* row = f.part + (long long)c * f.pstride;
    double pv[kFoldPer];
#pragma unroll
    for (int i = 0; i < kFoldPer; ++i)
        if (i * kFoldLanes < f.nchunks) pv[i] = row[min(l + i * kFoldLanes, f.nchunks - 1)];
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < kFoldPer; ++i)
        if (l + i * kFoldLanes < f.nchunks) sum += pv[i];
#pragma unroll
    for (int off = kFoldLanes / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, kFoldLanes);
    if (l == 0) f.hsum[c] = sum;
}

// Second part (hs published): the new B entry and the normalization, the common case of
// classical Gram-Schmidt (|r - B h|^2 = |r|^2 - |h|^2 >= |r|^2 / 2 and above the
// breakdown threshold), the same arithmetic as the reduction kernel in every thread.
// Returns false when the vector needs a DGKS pass or a fresh direction.
__device__ __forceinline__ bool fold_finish(const FoldRed& f, int ncols, double* hs, double bnorm, double& coef,
                                            double& scale) {
    const int tid = threadIdx.x;
    const double hh = sumsq_allwave(hs, ncols);
    const double rr = hs[ncols];
    if (f.full) {
        for (int c = tid; c < ncols; c += kFusedThreads) hs[c] = 0.0;
        lds_barrier();
        coef = 0.0;
        scale = 0.0;
        return true;
    }
    const double a2 = rr - hh;
    if (!(a2 >= 0.5 * rr && sqrt(a2) > f.tol_bd * bnorm)) return false;
    coef = sqrt(a2);
    scale = 1.0 / coef;
    return true;
}

template <int EPT, typename F1 = FftGeneric, bool FOLD = false>
__global__ __launch_bounds__(kFusedThreads) void k_p1_update(ConvGeom g, P1Seg a, float2* __restrict__ T1) {
    const double stopv = g.stop ? *g.stop : 0.0;  // tested once the first loads are in flight
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x;
    double pv[FOLD ? kFoldPer : 1];
    double bnorm = 0.0;
    const bool presummed = FOLD && a.fold.presummed;
    if constexpr (FOLD) {
        if (!presummed) fold_load(a.fold, a.ncols, tid, pv);
        bnorm = a.fold.bn[a.fold.par];
    }
    const int CB = g.CB, M1 = g.M1, M2 = g.M2, ss = M1 + 1;
    const int S = a.lay.S;
    float2* buf = smem;                                                   // CB x (M1 + 1)
    float2* tw = buf + CB * ss;                                           // M1
    double* red = reinterpret_cast<double*>(smem + fused_fft_lds_words(g));  // kFusedThreads x 4
    double* hs = red + 4 * kFusedThreads;                                 // ncols + 1
    SegSrc* src = reinterpret_cast<SegSrc*>(hs + ((a.ncols + 2) & ~1));   // 2 * CB
    const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
    const int ncb = min(CB, M2 - c0);
    // Every global load of the preamble is issued before the first LDS write: a write of
    // a loaded value waits for all loads issued before it (the counter is in order).
    const int wave0 = tid & ~63;  // (whole waves past the data skip their loads)
    float2 twv[kTwPer];           // M1 <= kTwPer * kFusedThreads
#pragma unroll
    for (int i = 0; i < kTwPer; ++i)
        if (wave0 + i * kFusedThreads < M1) twv[i] = g.tw1[min(tid + i * kFusedThreads, M1 - 1)];
    // h (ncols values), or with presummed column sums h and |r|^2 (ncols + 1)
    double hv[kHPer];  // ncols + 1 <= kHPer * kFusedThreads
    const int nh = FOLD ? (presummed ? a.ncols + 1 : 0) : a.ncols;
    const double* hsrc = FOLD ? a.fold.hsum : a.h;
    if (nh > 0) {
#pragma unroll
        for (int i = 0; i < kHPer; ++i)
            if (wave0 + i * kFusedThreads < nh) hv[i] = hsrc[min(tid + i * kFusedThreads, nh - 1)];
    }
    // x at every slot of the 2*ncb source segments, FP64.  The float4 groups are
    // split over the threads; when there are few of them the columns are split too,
    // over slices of threads whose sums meet in LDS in a fixed order.  A thread's
    // first columns are loaded before the barrier that publishes h.
    const int gps = S / 4;  // float4 groups per segment
    const int nf = 2 * ncb * gps;
    const int nf64 = (nf + 63) & ~63;
    const int nslice = min(16, kFusedThreads / nf64);  // 0 or 1: no column split
    const int slice = nslice >= 2 ? tid / nf64 : 0, f0 = nslice >= 2 ? tid % nf64 : tid;
    const int nsl_ = nslice >= 2 ? nslice : 1;
    // r at the group this thread finishes first (f = tid) and the first kUpdPre columns of
    // its accumulation group.  The loads are unconditional, at a group and a column clamped
    // into bounds (unused values are never read): branches around them would make the
    // compiler wait for each one in turn.
    float4 pre[kUpdPre];
#pragma unroll
    for (int u = 0; u < kUpdPre; ++u) pre[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    bool pre_ok = false;
    float4 rpre;  // read only where tid < nf, at the slots holding elements
    {
        const int f = min(tid, nf - 1), sg = f / gps;
        const SegSrc d = seg_source(a, M2, S, c0, sg);
        rpre = *reinterpret_cast<const float4*>(a.r + d.pos + 4 * (f - sg * gps));
    }
    if (a.ncols > 0) {
        const bool mine = slice < nsl_ && f0 < nf;
        const int f = mine ? f0 : 0, sg = f / gps;
        const SegSrc d = seg_source(a, M2, S, c0, sg);
        pre_ok = mine && 4 * (f - sg * gps) < d.cnt;
        const long long p = d.pos + 4LL * (f - sg * gps);
        // (clamped, not skipped: a branch around each load would have the compiler convert
        // the value inside it, waiting for every load in turn)
#pragma unroll
        for (int u = 0; u < kUpdPre; ++u) {
            const int c = min(slice + u * nsl_, a.ncols - 1);
            pre[u] = *reinterpret_cast<const float4*>(a.basis + (long long)c * a.ld + p);
        }
    }
    const double scale_in = FOLD ? 0.0 : *a.scale;
#pragma unroll
    for (int i = 0; i < kTwPer; ++i)
        if (tid + i * kFusedThreads < M1) tw[tid + i * kFusedThreads] = twv[i];
    for (int idx = tid; idx < CB * ss; idx += kFusedThreads) buf[idx] = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < kHPer; ++i)
        if (tid + i * kFusedThreads < nh) hs[tid + i * kFusedThreads] = hv[i];
    if (tid < 2 * ncb) src[tid] = seg_source(a, M2, S, c0, tid);
    double scale;
    if constexpr (FOLD) {
        if (!presummed) fold_sums(a.fold, a.ncols, hs, tid, pv);
        if (stopv != 0.0) return;
        lds_barrier();
        double coef;
        if (!fold_finish(a.fold, a.ncols, hs, bnorm, coef, scale)) {
            // every workgroup takes this branch (same sums); a stopped solve is left alone
            if (blockIdx.x == 0 && tid == 0) *a.fold.fail = kDoneFallback;
            return;
        }
        if (blockIdx.x == 0 && tid == 0) {
            *a.fold.coef_out = coef;
            a.fold.bn[a.fold.par ^ 1] = (a.fold.track && coef > bnorm) ? coef : bnorm;
            if (a.fold.snap) {
                a.fold.snap[0] = 0.0;
                a.fold.snap[1] = 0.0;
            }
        }
    } else {
        scale = scale_in;
        if (stopv != 0.0) return;
        lds_barrier();
    }
    if (nslice >= 2) {
        const int f = f0;
        if (slice < nslice && f < nf) {
            double x[4];
            fused_accumulate(a, hs, src, gps, f, slice, nslice, x, pre, pre_ok);
            for (int u = 0; u < 4; ++u) red[4 * tid + u] = x[u];
        }
        lds_barrier();
        if (tid < nf) {
            double x[4] = {0.0, 0.0, 0.0, 0.0};
            for (int sl = 0; sl < nslice; ++sl)
                for (int u = 0; u < 4; ++u) x[u] += red[4 * (sl * nf64 + tid) + u];
            fused_finish_group(a, src, gps, tid, x, scale, buf, ss, rpre);
        }
    } else {
        for (int f = tid; f < nf; f += kFusedThreads) {
            double x[4];
            fused_accumulate(a, hs, src, gps, f, 0, 1, x, pre, f == tid && pre_ok);
            const float4 rv = f == tid ? rpre : fused_load_r(a, src[f / gps], gps, f, f / gps);
            fused_finish_group(a, src, gps, f, x, scale, buf, ss, rv);
        }
    }
    lds_barrier();
    fft_run_waves<-1, EPT>(F1{}, buf, g.st1, CB, ss, tw, tid, kFusedThreads);
    for (int idx = tid; idx < CB * M1; idx += kFusedThreads) {
        const int c = idx % CB, k1 = idx / CB, n2 = c0 + c;
        if (n2 < M2) T1[(long long)k1 * M2 + n2] = cmul(buf[c * ss + k1], twiddle_mp(g, (long long)n2 * k1));
    }
}

// Start vector p_0 of Algorithm 1 in the segment layout: element i of a seeded
// standard normal stream at its slot, zero in the padding slots.
__global__ void k_start_seg(float* r, SegLay lay, unsigned long long seed) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lay.len) return;
    const long long i = seg_natural(lay, t / lay.S, t % lay.S);
    r[t] = i >= 0 ? gauss(seed, 0, i) : 0.0f;
}

// Ritz vectors out[i*ldo + nat(t)] = sum_c basis[c][t] P[c*k + i] of a basis in the
// segment layout: 64 stored slots and TILE triples per workgroup (the smallest tile that
// holds k, so that k <= 32 takes one pass over the basis), with the coefficients in LDS;
// its four waves take every fourth column (eight loads in flight each) and wave 0 adds
// the four partial sums in a fixed order.  Padding slots write nothing.
constexpr int kRitzSegWaves = 4;
template <int kRitzSegTile>
__global__ __launch_bounds__(64 * kRitzSegWaves) void k_ritz_seg(const float* __restrict__ basis, long long ld,
                                                                 int ncols, const double* __restrict__ P, int k,
                                                                 float* __restrict__ out, long long ldo, SegLay lay) {
    extern __shared__ double ps[];  // ncols x kRitzSegTile, then (waves - 1) x 64 x kRitzSegTile
    double* red = ps + (long long)ncols * kRitzSegTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = blockIdx.y * kRitzSegTile;
    const int kt = min(kRitzSegTile, k - i0);
    for (int idx = tid; idx < ncols * kRitzSegTile; idx += 64 * kRitzSegWaves) {
        const int c = idx / kRitzSegTile, i = idx - c * kRitzSegTile;
        ps[idx] = i < kt ? P[(long long)c * k + i0 + i] : 0.0;
    }
    lds_barrier();
    const long long t = (long long)blockIdx.x * 64 + lane;
    const bool valid = t < lay.len;
    const long long tc = valid ? t : 0;  // in-bounds slot for the loads of the tail lanes
    double acc[kRitzSegTile];
#pragma unroll
    for (int i = 0; i < kRitzSegTile; ++i) acc[i] = 0.0;
    constexpr int kStep = kRitzSegWaves;
    int c = wave;
    for (; c + 7 * kStep < ncols; c += 8 * kStep) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = basis[(long long)(c + u * kStep) * ld + tc];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int i = 0; i < kRitzSegTile; ++i) acc[i] += (double)x[u] * ps[(c + u * kStep) * kRitzSegTile + i];
    }
    for (; c < ncols; c += kStep) {
        const double x = basis[(long long)c * ld + tc];
#pragma unroll
        for (int i = 0; i < kRitzSegTile; ++i) acc[i] += x * ps[c * kRitzSegTile + i];
    }
    if (wave > 0) {
#pragma unroll
        for (int i = 0; i < kRitzSegTile; ++i) red[((wave - 1) * 64 + lane) * kRitzSegTile + i] = acc[i];
    }
    lds_barrier();
    if (wave != 0 || !valid) return;
    const long long nat = seg_natural(lay, t / lay.S, t % lay.S);
    if (nat < 0) return;
#pragma unroll
    for (int i = 0; i < kRitzSegTile; ++i) {
        double v = acc[i];
        for (int w = 1; w < kRitzSegWaves; ++w) v += red[((w - 1) * 64 + lane) * kRitzSegTile + i];
        if (i < kt) out[(long long)(i0 + i) * ldo + nat] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// launchers

static int fused_ept(long long elems) {
    const long long e = (elems + kFusedThreads - 1) / kFusedThreads;
    if (e <= 4) return 4;
    return 8;  // CB * M1 <= 8192
}

size_t fused_p3_lds(const ConvGeom& g, const SegLay& lay) {
    return sizeof(float2) * (size_t)fused_fft_lds_words(g) + sizeof(float) * 2 * (size_t)g.CB * lay.S;
}

size_t fused_p1_lds(const ConvGeom& g, int ncols) {
    return sizeof(float2) * (size_t)fused_fft_lds_words(g) +
           sizeof(double) * (4 * (size_t)kFusedThreads + ((ncols + 2) & ~1)) + sizeof(SegSrc) * 2 * (size_t)g.CB;
}

hipError_t launch_p3_project(const ConvGeom& g, const float2* T2, const P3Seg& a, hipStream_t s) {
    const dim3 grid((g.M2 + g.CB - 1) / g.CB);
    const size_t lds = fused_p3_lds(g, a.lay);
    if (fused_ept((long long)g.CB * g.M1) != 4)
        SSA_LAUNCH(k_p3_project<8>, grid, dim3(kFusedThreads), lds, s, g, T2, a);
    else if (FftPlanA::matches(g.st1))
        SSA_LAUNCH((k_p3_project<4, FftPlanA>), grid, dim3(kFusedThreads), lds, s, g, T2, a);
    else if (FftPlanB::matches(g.st1))
        SSA_LAUNCH((k_p3_project<4, FftPlanB>), grid, dim3(kFusedThreads), lds, s, g, T2, a);
    else
        SSA_LAUNCH(k_p3_project<4>, grid, dim3(kFusedThreads), lds, s, g, T2, a);
    return hipGetLastError();
}

template <bool FOLD>
static void launch_p1_variant(const ConvGeom& g, const P1Seg& a, float2* T1, hipStream_t s) {
    const dim3 grid((g.M2 + g.CB - 1) / g.CB);
    const size_t lds = fused_p1_lds(g, a.ncols);
    if (fused_ept((long long)g.CB * g.M1) != 4)
        SSA_LAUNCH((k_p1_update<8, FftGeneric, FOLD>), grid, dim3(kFusedThreads), lds, s, g, a, T1);
    else if (FftPlanA::matches(g.st1))
        SSA_LAUNCH((k_p1_update<4, FftPlanA, FOLD>), grid, dim3(kFusedThreads), lds, s, g, a, T1);
    else if (FftPlanB::matches(g.st1))
        SSA_LAUNCH((k_p1_update<4, FftPlanB, FOLD>), grid, dim3(kFusedThreads), lds, s, g, a, T1);
    else
        SSA_LAUNCH((k_p1_update<4, FftGeneric, FOLD>), grid, dim3(kFusedThreads), lds, s, g, a, T1);
}

hipError_t launch_p1_update(const ConvGeom& g, const P1Seg& a, float2* T1, hipStream_t s) {
    if (a.fold.part)
        launch_p1_variant<true>(g, a, T1, s);
    else
        launch_p1_variant<false>(g, a, T1, s);
    return hipGetLastError();
}

hipError_t launch_fold_sums(const FoldRed& f, int ncols, hipStream_t s) {
    const int per = 64 / kFoldLanes;
    SSA_LAUNCH(k_fold_sums, dim3((unsigned)((ncols + per) / per)), dim3(64), 0, s, f, ncols);
    return hipGetLastError();
}

hipError_t launch_start_seg(float* r, const SegLay& lay, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(k_start_seg, dim3((unsigned)((lay.len + 255) / 256)), dim3(256), 0, s, r, lay, seed);
    return hipGetLastError();
}

template <int TILE>
static hipError_t launch_ritz_seg_t(const float* basis, long long ld, int ncols, const double* P, int k, float* out,
                                    long long ldo, const SegLay& lay, hipStream_t s) {
    const dim3 grid((unsigned)((lay.len + 63) / 64), (unsigned)((k + TILE - 1) / TILE));
    const size_t lds = sizeof(double) * ((size_t)ncols + (kRitzSegWaves - 1) * 64) * TILE;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    SSA_LAUNCH(k_ritz_seg<TILE>, grid, dim3(64 * kRitzSegWaves), lds, s, basis, ld, ncols, P, k, out, ldo, lay);
    return hipGetLastError();
}

hipError_t launch_ritz_seg(const float* basis, long long ld, int ncols, const double* P, int k, float* out,
                           long long ldo, const SegLay& lay, hipStream_t s) {
    if (k <= 8) return launch_ritz_seg_t<8>(basis, ld, ncols, P, k, out, ldo, lay, s);
    if (k <= 12) return launch_ritz_seg_t<12>(basis, ld, ncols, P, k, out, ldo, lay, s);
    if (k <= 16) return launch_ritz_seg_t<16>(basis, ld, ncols, P, k, out, ldo, lay, s);
    if (k <= 20) return launch_ritz_seg_t<20>(basis, ld, ncols, P, k, out, ldo, lay, s);
    if (k <= 24) return launch_ritz_seg_t<24>(basis, ld, ncols, P, k, out, ldo, lay, s);
    return launch_ritz_seg_t<32>(basis, ld, ncols, P, k, out, ldo, lay, s);
}

hipError_t set_fused_attributes() {
    hipError_t e = hipSuccess;
    auto allow = [&](const void* f) {
        const hipError_t e2 = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e2 != hipSuccess) e = e2;
    };
    allow(reinterpret_cast<const void*>(k_p3_project<4>));
    allow(reinterpret_cast<const void*>(k_p3_project<8>));
    allow(reinterpret_cast<const void*>(k_p1_update<4>));
    allow(reinterpret_cast<const void*>(k_p1_update<8>));
    allow(reinterpret_cast<const void*>(k_p3_project<4, FftPlanA>));
    allow(reinterpret_cast<const void*>(k_p3_project<4, FftPlanB>));
    allow(reinterpret_cast<const void*>(k_p1_update<4, FftPlanA>));
    allow(reinterpret_cast<const void*>(k_p1_update<4, FftPlanB>));
    allow(reinterpret_cast<const void*>(k_p1_update<4, FftGeneric, true>));
    allow(reinterpret_cast<const void*>(k_p1_update<8, FftGeneric, true>));
    allow(reinterpret_cast<const void*>(k_p1_update<4, FftPlanA, true>));
    allow(reinterpret_cast<const void*>(k_p1_update<4, FftPlanB, true>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<8>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<12>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<16>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<20>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<24>));
    allow(reinterpret_cast<const void*>(k_ritz_seg<32>));
    return e;
}

}  // namespace ssa
