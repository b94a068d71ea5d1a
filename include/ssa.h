/*
 * ssa.h -- C ABI of the MI355X (gfx950) fast Basic SSA library.
 *
 * Method: Korobeynikov, "Computation- and Space-Efficient Implementation of
 * SSA".  Given a real series F = (f_1..f_N) and a window 1 < L < N
 * (Sec. 2), the library computes the k leading singular triples
 * (sigma_i, u_i, v_i) of the L x K trajectory matrix X (K = N - L + 1,
 * X[i][j] = f_{i+j}, Sec. 2.1) by Golub-Kahan-Lanczos bidiagonalization
 * (Sec. 3.1, Algorithm 1) with full reorthogonalization (Sec. 3.2.2), where
 * every product X v and X^T u is a circular convolution of the series
 * computed by FFT (Sec. 4, Algorithms 2 and 3) so X is never formed; and it
 * turns groups of triples back into series by FFT rank-1 Hankelization
 * (Sec. 5, Algorithm 4; Sec. 2.3-2.4 for grouping / diagonal averaging).
 *
 * Conventions shared by every entry point:
 *  - Indices are 0-based.  Device pointers ("_dev") are HIP device memory on
 *    the current device, owned by the caller; the library never allocates
 *    device memory.  Host pointers are ordinary host memory.
 *  - Work is enqueued on the stream given to ssa_plan_bind, in call order, and
 *    the calls return as soon as their work is enqueued; outputs are valid once
 *    the stream has run it.  ssa_truncated_svd is the exception in one respect:
 *    the stopping test runs on the device, but the host must learn its answer
 *    to stop enqueuing Lanczos steps, so the call waits for the test of each
 *    check point (one check point behind the steps it has enqueued) and reads
 *    back that test's small record -- never the Lanczos scalars.  With thick
 *    restart (ssa_opts.restart_keep) the projected matrix is solved on the
 *    host and the call returns after its result is complete.
 *  - A plan (and its workspace) may be used by one stream at a time.
 *    Distinct plans are independent.
 *  - Return values: 0 success; positive = warning, results written;
 *    negative = error, nothing enqueued (argument errors are detected
 *    before any work is enqueued).
 *  - Floating point: series input FP64; FFTs, matvecs and stored Lanczos
 *    vectors FP32; Lanczos scalars (alpha, beta), reorthogonalization inner
 *    products, norms and the small bidiagonal SVD FP64.
 */
#ifndef SSA_H
#define SSA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssa_plan_s* ssa_plan;

enum ssa_status {
    SSA_OK = 0,
    SSA_WARN_NOT_CONVERGED = 1, /* Krylov dimension cap reached before the stopping rule  */
    SSA_WARN_BREAKDOWN = 2,     /* converged, but an alpha or beta vanished on the way (the
                                   series has rank below the steps taken, or the Krylov space
                                   was exhausted): Algorithm 1 continued from a random vector
                                   orthogonal to the basis, and triples past the rank have
                                   sigma = 0 with arbitrary orthonormal vectors              */
    SSA_EINVAL = -1,            /* invalid argument (sizes, null pointers, group members) */
    SSA_ENOMEM = -2,            /* workspace missing or smaller than required             */
    SSA_ENONFINITE = -3,        /* the series holds NaN or Inf                            */
    SSA_EDEVICE = -4,           /* a HIP runtime call failed                              */
    SSA_EMISMATCH = -5,         /* N or L differ from the plan                            */
    SSA_ESTATE = -6             /* call order violated (e.g. matvec before embed)         */
};

/* Solver options; zero-initialized fields take the defaults shown. */
typedef struct {
    int d_max;              /* Krylov dimension cap (Sec. 3.3, d); default min(L,K,8k+32,1024) */
    int check_every;        /* Lanczos steps between stopping tests; default 4                 */
    double tol;             /* stop when every residual bound <= tol * max(omega_i, 1e-5 omega_1)
                               and the k Ritz values moved < 10 tol relative; default 1e-8   */
    unsigned long long seed;/* seed of the random start vector p_0 (Algorithm 1); default 1    */
    int fft_m1;             /* FFT schedule override: first factor M1 of M/2 = M1*M2 (must
                               divide M/2, both factors <= 4096); 0 = automatic              */
    int fft_cb;             /* columns per workgroup in FFT passes 1 and 3 (1..64); 0 = auto */
    int restart_keep;       /* thick restart (Sec. 3.3, restarting schemes): when the basis
                               reaches d_max columns without convergence, keep this many
                               Ritz pairs and continue, at most 64 times.  Needs
                               k_max <= restart_keep <= d_max - 2 and d_max <= 512 (unless
                               d_max >= min(L, K), when no restart can occur); 0 = off,
                               the plain Algorithm 1 that stops at d_max.  Single-series
                               solver only.                                               */
    int reorth;             /* 0: full reorthogonalization of both bases (Sec. 3.2, FRO);
                               1: one-sided (Simon and Zha): only the basis of length
                               min(L, K) is reorthogonalized, the other keeps the
                               three-term recurrence alone (half the Gram-Schmidt traffic).
                               One-sided cannot be combined with restart_keep.            */
    long long fft_mp;       /* FFT length override: M/2 = M' for the products and the
                               Hankelization (Sec. 4.2: any M >= N gives the exact
                               correlation).  Must be >= ceil(N/2), 7-smooth and split
                               into two factors <= 4096; 0 = the smallest such M'.  The
                               schedule tuner (ssa_tune_fft) picks it by measurement.    */
    int unfused;            /* 1: run each Lanczos half-step as six launches (pass 1, 2, 3,
                               projection, reduction, update) with the bases in natural
                               order; 2: the fused four-launch half-step (pass 1 with the
                               update, pass 2, pass 3 with the projection, reduction);
                               0 = fused wherever it applies (1D, no thick restart,
                               max(L, K) <= 2^20), with each reduction folded into the
                               next pass-1 launch (three launches) where pass 3 has at
                               most 256 workgroups.  A folded solve that meets a DGKS
                               pass or a breakdown restarts as four launches.  1 gives
                               the same results up to rounding order, 2 the same bits as
                               a folded solve that did not restart; an A/B switch.       */
} ssa_opts;

/* Per-solve report, filled by ssa_truncated_svd. */
typedef struct {
    int steps;         /* Lanczos steps d whose bidiagonal B_d gave the result (with thick
                          restarts: all steps of all cycles)                                */
    int converged;     /* 1 if the stopping rule held, 0 if d_max was reached                */
    int restarts;      /* vanishing alpha/beta replaced by fresh random directions           */
    int dgks_passes;   /* second Gram-Schmidt passes triggered by the DGKS criterion          */
    int steps_run;     /* Lanczos steps executed (>= steps: the stopping test of one check
                          point overlaps the next steps, which are then discarded)           */
    double resid[64];  /* residual bounds alpha_{d+1} |P[d+1,i]| of the first min(k,64) triples */
    int thick_restarts;/* restart cycles performed (ssa_opts.restart_keep)                   */
    int status;        /* the call's return value (SSA_OK or a warning; errors fill nothing) */
    int half_step_launches; /* launches per Lanczos half-step the result came from: 3 (each
                          reduction folded into the next pass-1 launch), 4 (the reduction as
                          its own launch; also where a folded solve met a DGKS pass or a
                          breakdown and was restarted), or 6 (ssa_opts.unfused = 1, 2D,
                          thick restart, max(L, K) > 2^20)                                   */
} ssa_info;

/* Sizes chosen by a plan (reported for tests and benchmarks). */
typedef struct {
    long long N, L, K;  /* as requested (L > K is accepted; it is solved transposed)   */
    long long M;        /* FFT length: even, >= N (any M >= N is exact, Sec. 4.3)        */
    long long M1, M2;   /* M/2 = M1 * M2, the two passes of the half-length complex FFT */
    int d_max, k_max;
    size_t workspace_bytes;
    int cb;             /* columns per workgroup of FFT passes 1 and 3                   */
} ssa_plan_desc;

/*
 * ssa_embed_plan -- Sec. 2.1 / Sec. 4.3: size everything for a series of
 * length N and window L, solving for at most k_max triples.
 *   N > 2, 1 < L < N, 1 <= k_max <= min(L, K); opts may be NULL.
 *   *workspace_bytes receives the device workspace size the plan needs.
 *   *out receives a host-side plan object (free with ssa_plan_destroy).
 * Errors: SSA_EINVAL (sizes, null out pointers).
 */
int ssa_embed_plan(long long N, long long L, int k_max, const ssa_opts* opts,
                   size_t* workspace_bytes, ssa_plan* out);

/*
 * ssa_embed_plan_2d -- 2D-SSA (named in Sec. 1 and Sec. 3.3 as the case whose
 * trajectory matrix is Hankel with Hankel blocks): an Nx x Ny array F
 * (row-major, F[i][j] at i * Ny + j) with an Lx x Ly window.  The trajectory
 * matrix is X[(a, b), (c, d)] = F[a + c][b + d], rows a * Ly + b (a < Lx,
 * b < Ly), columns c * Ky + d (c < Kx = Nx - Lx + 1, d < Ky = Ny - Ly + 1).
 * The plan is then used like a 1D plan of N = Nx Ny, L = Lx Ly, K = Kx Ky:
 * ssa_truncated_svd takes that N and L (the array flattened row by row) and
 * returns U ((Lx Ly) x k: each u_i an Lx x Ly array row by row) and V
 * ((Kx Ky) x k); ssa_matvec takes and returns such compressed vectors;
 * ssa_reconstruct writes m arrays of Nx x Ny (row-major), the 2D diagonal
 * averaging (mean over a + c = i, b + d = j).  Products and averaging run on
 * the row-pitch-Ny flattening, where X is a row/column selection of the 1D
 * Hankel matrix of the flattened array, so the FFT length covers Nx Ny.
 *   1 <= Lx <= Nx, 1 <= Ly <= Ny, Lx Ly >= 2, Kx Ky >= 2,
 *   1 <= k_max <= min(Lx Ly, Kx Ky).
 * Errors: SSA_EINVAL.
 */
int ssa_embed_plan_2d(long long Nx, long long Ny, long long Lx, long long Ly, int k_max, const ssa_opts* opts,
                      size_t* workspace_bytes, ssa_plan* out);

/*
 * ssa_plan_bind -- attach caller-owned device workspace (>= workspace_bytes,
 * 256-byte aligned) and a HIP stream (hipStream_t passed as void*, NULL =
 * the default stream).  Errors: SSA_EINVAL (null plan/workspace, bad
 * alignment), SSA_ENOMEM (too small).
 */
int ssa_plan_bind(ssa_plan plan, void* workspace_dev, size_t bytes, void* hip_stream);

/*
 * ssa_embed -- Algorithm 2, steps 1-2 (done once per series): the spectrum
 * of the zero-padded series, stored in the workspace as the operator that
 * every later X v / X^T u applies.  series_dev: N doubles.
 * Errors: SSA_EINVAL, SSA_ENOMEM (unbound plan).
 */
int ssa_embed(ssa_plan plan, const double* series_dev);

/*
 * ssa_matvec -- Algorithms 2 / 3: y = X x (transpose = 0; x has K entries,
 * y gets L) or y = X^T x (transpose = 1; x has L entries, y gets K), as an
 * FFT convolution with the embedded series.  FP32 vectors, device memory.
 * Errors: SSA_EINVAL, SSA_ESTATE (no ssa_embed yet).
 */
int ssa_matvec(ssa_plan plan, int transpose, const float* x_dev, float* y_dev);

/*
 * ssa_matvec_static -- the product of ssa_matvec for callers that cannot
 * allocate device memory or bind a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  One call computes the
 * operator of the series (ssa_embed) and then y = X x (transpose = 0; x has
 * K = N - L + 1 entries, y gets L) or y = X^T x (transpose = 1; x has L, y gets
 * K), with the FFT schedule ssa_embed_plan picks without options, so y has the
 * same bits as ssa_embed + ssa_matvec on such a plan.
 *   series_dev: N doubles; x_dev, y_dev: FP32 device vectors, caller-owned.
 *   hip_stream: hipStream_t as void* (NULL = the default stream).
 * Every intermediate (twiddle tables, the series' spectral operator, two FFT
 * buffers) lives in a static device array of the library, 16.25 MiB per GPU,
 * held until the process ends; the call allocates nothing.  Limit: N <= 2^20.
 * All calls on one GPU share that array and it keeps the last call's contents:
 * calls that overlap on one GPU (different streams or threads) race and must be
 * serialized by the caller.  The series is not checked for NaN/Inf (no host
 * synchronization); non-finite input gives non-finite output.
 * Asynchronous on hip_stream.  Errors: SSA_EINVAL (null pointers, N <= 2,
 * L outside (1, N)), SSA_ENOMEM (N > 2^20), SSA_EDEVICE.
 */
int ssa_matvec_static(const double* series_dev, long long N, long long L, int transpose,
                      const float* x_dev, float* y_dev, void* hip_stream);

/*
 * ssa_truncated_svd -- Sec. 2.2 via Sec. 3 + 4: the k leading singular
 * triples of X, sigma descending.
 *   series_dev: N doubles (device).  N, L must equal the plan's.
 *   sigma_dev: k doubles; U_dev: L x k floats column-major (u_i at
 *   U_dev + i*L); V_dev: K x k floats column-major (v_i at V_dev + i*K).
 *   info: optional host struct (may be NULL).
 * Returns SSA_OK, SSA_WARN_NOT_CONVERGED, SSA_WARN_BREAKDOWN, or an error:
 * SSA_EINVAL (k outside [1, k_max]), SSA_EMISMATCH, SSA_ENOMEM (unbound
 * plan), SSA_ENONFINITE (series holds NaN/Inf, found on the device by the
 * first stopping test; outputs untouched), SSA_EDEVICE.
 * Without thick restart: info is complete on return, sigma_dev/U_dev/V_dev
 * once the plan's stream has run the enqueued work (stream-ordered).  With
 * thick restart the stream is synchronized before returning.
 */
int ssa_truncated_svd(ssa_plan plan, const double* series_dev, long long N, long long L, int k,
                      double* sigma_dev, float* U_dev, float* V_dev, ssa_info* info);

/*
 * ssa_reconstruct -- Sec. 2.3-2.4 with Sec. 5: for each group g of triple
 * indices (CSR on the host: group_offsets[m+1], group_members[]), the
 * diagonal average of sum_{i in g} sigma_i u_i v_i^T, computed as FFT linear
 * convolutions of u_i and v_i scaled by 1/(number of entries on each
 * antidiagonal).  Groups may overlap; each is an independent linear map.
 *   sigma_dev, U_dev, V_dev: as returned by ssa_truncated_svd with k triples.
 *   out_dev: m x N floats, row-major (group g at out_dev + g*N).
 * Errors: SSA_EINVAL (k outside [1, k_max], member outside [0,k), member
 * repeated within a group, m < 1), SSA_ENOMEM (unbound plan).
 */
int ssa_reconstruct(ssa_plan plan, const double* sigma_dev, const float* U_dev,
                    const float* V_dev, int k, const int* group_offsets,
                    const int* group_members, int m, float* out_dev);

/*
 * Many independent series solved together (the batched path).  The series
 * advance in lockstep, one launch per Lanczos half-step for the whole batch
 * with one workgroup per series.  Each workgroup runs Algorithm 1 for its
 * series: the FFT products of Algorithms 2/3 and classical Gram-Schmidt
 * reorthogonalization (Sec. 3.2.2), all in LDS.  At check points the stopping
 * test on B_j runs on the device (eqs. lbdiagm1/lbdiagm2).  At the end come the
 * Ritz triples and the rank-1 Hankelization of every triple (Algorithm 4).
 * A series' result depends only on the series, its key and the seed: it is
 * the same alone and inside any batch.
 */
typedef struct ssa_batch_s* ssa_batch;

/*
 * ssa_batch_plan -- host-side engine for up to max_series series per solve.
 * Each series has length 3 <= N <= n_max (n_max <= 20480) and up to
 * k_max <= 32 triples.  opts as for ssa_embed_plan; d_max is capped at 320;
 * fft_m1/fft_cb/fft_mp do not apply (each series' FFT is one workgroup's); reorth
 * applies to every series; restart_keep must be 0.
 * *workspace_bytes: enough for max_series series of length n_max with
 * L = n_max/2 and k = k_max.  ssa_batch_workspace gives the exact figure for
 * given series.  Errors: SSA_EINVAL.
 */
int ssa_batch_plan(long long n_max, int k_max, int max_series, const ssa_opts* opts,
                   size_t* workspace_bytes, ssa_batch* out);

/*
 * ssa_batch_workspace -- device workspace bytes that ssa_batch_solve needs for
 * these series (same host arrays as ssa_batch_solve).  Errors: SSA_EINVAL.
 */
int ssa_batch_workspace(ssa_batch batch, int nseries, const long long* offsets, const int* L,
                        const int* k, size_t* bytes);

/* ssa_batch_bind -- as ssa_plan_bind, for a batch engine (workspace 256-byte aligned). */
int ssa_batch_bind(ssa_batch batch, void* workspace_dev, size_t bytes, void* hip_stream);

/*
 * ssa_batch_solve -- the k_s leading triples of every series s and, if
 * recon_dev is not NULL, its k_s elementary reconstructed series.
 *   series_dev: all series concatenated (FP64, device).
 *   offsets (host, nseries+1, offsets[0] = 0): series s is
 *     series_dev[offsets[s] .. offsets[s+1]).
 *   L (host, nseries): window lengths, 1 < L[s] < N_s.
 *   k (host, nseries): triples, 1 <= k[s] <= min(k_max, L[s], K_s).
 *   keys (host, nseries, may be NULL = 0..nseries-1): seed the start and
 *     restart vectors of each series.  A series with the same key gives the
 *     same bits alone and in any batch.
 *   Outputs (device), one block per series in input order:
 *     sigma_dev: k_s doubles, descending;
 *     U_dev: L_s*k_s floats (u_i at + i*L_s);
 *     V_dev: K_s*k_s floats (v_i at + i*K_s);
 *     recon_dev: N_s*k_s floats (elementary series i at + i*N_s);
 *     info_dev (may be NULL): 4 ints per series (steps d, converged,
 *       restarts, DGKS passes).
 * Asynchronous on the bound stream.  The host returns once every series has
 * finished its steps; the outputs are valid after the stream synchronizes.
 * Errors: SSA_EINVAL, SSA_ENOMEM (unbound, or the bound workspace is smaller
 * than ssa_batch_workspace), SSA_EDEVICE.
 */
int ssa_batch_solve(ssa_batch batch, int nseries, const double* series_dev, const long long* offsets,
                    const int* L, const int* k, const unsigned long long* keys, double* sigma_dev,
                    float* U_dev, float* V_dev, float* recon_dev, int* info_dev);

/* Kernel classes of the batch engine's optional timing. */
enum ssa_batch_prof_class {
    SSA_BPROF_INIT = 0,  /* spectra, twiddles, start vectors                      */
    SSA_BPROF_CONV,      /* FFT products (Algorithms 2/3), one launch per half-step */
    SSA_BPROF_CGS,       /* Gram-Schmidt steps (Sec. 3.2.2), one per half-step   */
    SSA_BPROF_CHECK,     /* stopping tests (eqs. lbdiagm1/lbdiagm2)              */
    SSA_BPROF_RITZ,      /* Ritz triples                                         */
    SSA_BPROF_HANKEL,    /* rank-1 Hankelization (Algorithm 4)                   */
    SSA_BPROF_NCLASSES
};

/*
 * ssa_batch_profile_enable -- from now on, bracket every launch of the classes
 * in class_mask (bit c = class c) with HIP events on the bound stream; clears
 * earlier counts.  0 stops timing.  Synchronizes the bound stream.
 */
int ssa_batch_profile_enable(ssa_batch batch, unsigned class_mask);

/*
 * ssa_batch_profile_read -- launches of class cls since the last enable and,
 * if the class is timed, the summed event-measured milliseconds (else -1).
 * Synchronizes the bound stream.  Errors: SSA_EINVAL, SSA_EDEVICE.
 */
int ssa_batch_profile_read(ssa_batch batch, int cls, long long* launches, double* ms);

/* ssa_batch_destroy -- free the host-side batch engine. */
void ssa_batch_destroy(ssa_batch batch);

/*
 * Continuous batching of SSA requests (served form).  A server owns a pool of
 * device memory (the caller's workspace, its HBM budget) and a number of
 * slots.  Submitted requests wait in one queue in arrival order and are
 * admitted, at the start of a tick, while a slot of their class is free and the
 * pool holds their region (a request whose class has no free slot lets later
 * requests of the other class pass; one the pool cannot hold stops admission
 * until it fits).  Every request's state stays in its pool region between ticks;
 * storage is O(d (L + K)) per request (Sec. 3.3 on the cost of the bases).
 * Short requests (N <= n_max) run on the batched engine: a tick enqueues one
 * Lanczos step (Algorithm 1 with the FFT products and Gram-Schmidt of the
 * batched path) for every admitted one, sets up the newly admitted ones and
 * finishes (Ritz triples, Algorithm 4) the ones whose stopping test held in the
 * previous tick.  Long requests (ssa_server_enable_long) run the single-series
 * solver on a plan bound to their region, each on a stream of its own: a tick
 * advances each by one check interval once its previous one has run, and
 * enqueues its Ritz triples and Hankelization once its device stopping test has
 * held.  A request gives the same result whatever else is in flight (its key
 * seeds its start vector).
 */
typedef struct ssa_server_s* ssa_server;

/*
 * ssa_server_create -- batched requests of length 3 <= N <= n_max (n_max <=
 * 20480), k <= k_max <= 32, at most `slots` of them in flight (longer ones:
 * ssa_server_enable_long); opts as for ssa_batch_plan.
 * workspace_dev (256-byte aligned, `bytes` long) is the device pool; the
 * library allocates no device memory.  Errors: SSA_EINVAL, SSA_ENOMEM (pool
 * too small for the slot tables).
 */
int ssa_server_create(long long n_max, int k_max, int slots, const ssa_opts* opts, void* workspace_dev,
                      size_t bytes, void* hip_stream, ssa_server* out);

/*
 * ssa_server_enable_long -- also serve requests with n_max < N <= n_long_max
 * (n_long_max <= 2^24), at most long_slots at a time.  Each is planned at
 * submission (ssa_embed_plan with the server's opts, its seed mixed with the
 * request key) and takes a pool region of the plan's workspace size.  Creates
 * one HIP stream, one event and a few pinned bytes per long slot.  Errors:
 * SSA_EINVAL, SSA_ESTATE (already enabled), SSA_EDEVICE.
 */
int ssa_server_enable_long(ssa_server server, long long n_long_max, int long_slots);

/*
 * ssa_server_create_stub -- a server whose executor is a stub, for tests of the
 * queue and of admission on machines without a GPU: no device memory, stream or
 * HIP call; the pool is pool_bytes of bookkeeping only; every admitted request
 * reports its test passed after `ticks` ticks and completes like a real one.
 * Submitted pointers are never dereferenced.
 */
int ssa_server_create_stub(long long n_max, int k_max, int slots, const ssa_opts* opts, size_t pool_bytes,
                           int ticks, ssa_server* out);

/* ssa_server_request_bytes -- pool bytes a request of this shape occupies. */
int ssa_server_request_bytes(ssa_server server, long long N, long long L, int k, size_t* bytes);

/*
 * ssa_server_submit -- queue a request.  series_dev (N FP64 values) and the
 * outputs (sigma_dev: k doubles; U_dev: L*k floats, u_i at + i*L; V_dev:
 * K*k floats; recon_dev: N*k floats or NULL; info_dev: 4 ints or NULL: steps,
 * converged (-1 for a long request whose series holds NaN or Inf), restarts,
 * DGKS passes) are device memory that must hold no pending work of other
 * streams at submission (a long request is solved on a stream of its own) and stay valid
 * until `id` is reported complete by ssa_server_step.  Errors: SSA_EINVAL,
 * SSA_ENOMEM (the request alone exceeds the pool).
 */
int ssa_server_submit(ssa_server server, long long id, unsigned long long key, const double* series_dev,
                      long long N, long long L, int k, double* sigma_dev, float* U_dev, float* V_dev,
                      float* recon_dev, int* info_dev);

/*
 * ssa_server_step -- one tick (see above); returns when the tick's work is
 * done on the device.  completed[0 .. *ncompleted) receives the ids of
 * requests whose outputs are complete (at most max_completed; the others are
 * reported by later ticks).  Errors: SSA_EINVAL, SSA_EDEVICE.
 */
int ssa_server_step(ssa_server server, long long* completed, int max_completed, int* ncompleted);

/* ssa_server_status -- requests queued, being solved, being finished; free pool bytes. */
int ssa_server_status(ssa_server server, int* queued, int* active, int* finalizing, size_t* pool_free_bytes);

/* ssa_server_destroy -- free the host-side server (waits for its stream). */
void ssa_server_destroy(ssa_server server);

/*
 * Structural-change detection (the H-matrix of Sec. "Detection of Structural
 * Changes", eq. g).  G[i * (N-T+1) + j] (row-major, FP64) is the
 * heterogeneity index of test window f[j .. j+T-1] against the eigenvector
 * span {U_i, i in I} of base window f[i .. i+B-1] (window length L): the share
 * of the test window's lagged-vector energy outside that span.  The base
 * windows' SSAs run together on the batched path.  I: host array of nI
 * 1-based triple indices, each <= 32.  Limits: L < B - 1, L <= T,
 * B <= 20480, B, T <= N, nI*L + L + 256 <= 40960.
 */
int ssa_hmatrix_workspace(long long N, long long B, long long T, long long L, const int* I, int nI,
                          size_t* bytes);

/*
 * ssa_hmatrix -- the H-matrix of series_dev (N FP64 values, device) into G_dev
 * ((N-B+1) x (N-T+1) doubles, device).  workspace_dev: 256-byte aligned, at
 * least ssa_hmatrix_workspace bytes.  Returns when G is complete.  Errors:
 * SSA_EINVAL, SSA_ENOMEM (workspace too small), SSA_EDEVICE.
 */
int ssa_hmatrix(const double* series_dev, long long N, long long B, long long T, long long L, const int* I,
                int nI, void* workspace_dev, size_t bytes, void* hip_stream, double* G_dev);

/*
 * Repeated realizations (Sec. "Bootstrap Confidence Intervals Construction").
 * series_dev holds R realizations of length N (row r at + r*N, FP64, device).
 * Each is reconstructed from its first d eigentriples, with window L
 * (Sec. 2.3-2.4, group {1..d}), on the batched path.  Per point n:
 *   mean_dev[n] = mean over r of G_r[n];
 *   var_dev[n]  = (R-1)-normalized variance;
 *   mse_dev[n]  = mean square error against truth_dev (optional: both NULL or both given).
 * A bootstrap confidence interval for the mean reconstruction follows as
 * mean +- z sqrt(var / R).  Limits: N <= 20480, d <= 32, d <= min(L, K).
 * Returns when the statistics are complete.
 */
int ssa_realizations_workspace(long long R, long long N, long long L, int d, size_t* bytes);
int ssa_realizations(const double* series_dev, long long R, long long N, long long L, int d,
                     const double* truth_dev, void* workspace_dev, size_t bytes, void* hip_stream,
                     double* mean_dev, double* var_dev, double* mse_dev);

/*
 * ssa_tune_workspace -- device bytes that ssa_tune_fft needs for a series of
 * length N with window L: the largest candidate plan (k_max = 1, d_max = 2)
 * plus four product vectors.  Errors: SSA_EINVAL (sizes, null bytes).
 */
int ssa_tune_workspace(long long N, long long L, size_t* bytes);

/*
 * ssa_tune_fft -- choose the FFT schedule of the products X v and X^T u
 * (Algorithms 2 and 3) by measurement.  Any M >= N gives the exact correlation
 * (Sec. 4.2), so the transform length M' = M/2 is free above ceil(N/2), and so
 * are its split M' = M1 * M2 and the columns per workgroup CB of passes 1 and 3.
 * Candidates: the automatic schedule; the 8 smallest 7-smooth M' in
 * [ceil(N/2), 1.25 ceil(N/2)] that split into factors in [16, 4096], each with
 * its 6 most balanced splits and CB in {1, 2, 4, 8} (CB * M1 <= 8192, CB <= M2).
 * Each candidate: a plan is created and bound to workspace_dev, series_dev is
 * embedded, 2 product pairs warm up, then 3 runs of reps pairs are timed with
 * HIP events on hip_stream (hipStream_t as void*, NULL = default stream); the
 * candidate's time is its fastest run per pair.  The product time does not
 * depend on the series' values.
 *   series_dev: N doubles on the device (read only).
 *   workspace_dev: >= ssa_tune_workspace bytes, 256-byte aligned, overwritten.
 *   best: its fft_mp, fft_m1 and fft_cb receive the fastest schedule (explicit
 *     values, never 0); its other fields are left as they are.
 *   us_best (may be NULL): microseconds per product pair of that schedule.
 *   rows/us (may be NULL when max_rows = 0): the first max_rows candidates
 *     timed, as {M', M1, CB} triples in rows and microseconds per pair in us;
 *     *nrows (may be NULL) receives the number of candidates timed.
 * Synchronizes hip_stream.  Errors: SSA_EINVAL (sizes, null pointers),
 * SSA_ENOMEM (workspace too small or misaligned), SSA_ENONFINITE (series),
 * SSA_EDEVICE.
 */
int ssa_tune_fft(long long N, long long L, const double* series_dev, void* workspace_dev, size_t bytes,
                 void* hip_stream, int reps, ssa_opts* best, double* us_best, int max_rows, long long* rows,
                 double* us, int* nrows);

/* ssa_plan_describe -- copy the plan's sizes into *desc. */
int ssa_plan_describe(ssa_plan plan, ssa_plan_desc* desc);

/* ssa_plan_destroy -- free the host-side plan (the workspace stays the caller's). */
void ssa_plan_destroy(ssa_plan plan);

/*
 * ssa_bidiag_ritz -- host utility (no device work): singular values of the
 * (d+1) x d lower bidiagonal B_d of Sec. 3.1 (alpha[1..d] on the diagonal,
 * beta[2..d+1] below it; arrays indexed as in Algorithm 1, alpha[d+1] used
 * for the residual bound of eq. lbdiagm2).  Writes the k largest values to
 * omega (descending); if resid is given, their residual bounds
 * alpha_{d+1} |P[d,i]|; if P and Q are given, the singular vectors
 * (P: (d+1) x k row-major, Q: d x k row-major).  This is the routine the
 * solver uses for its stopping test and Ritz vectors.
 */
int ssa_bidiag_ritz(const double* alpha, const double* beta, int d, int k, double* omega,
                    double* resid, double* P, double* Q);

/*
 * ssa_dense_ritz -- host utility (no device work): the k largest singular
 * triples of a dense nr x nc matrix A (row-major, nr >= nc >= 1, k >= 1):
 * omega (k, descending), P (nr x k row-major, left vectors), Q (nc x k
 * row-major, right vectors); entries beyond min(k, nc) are zero.  Householder
 * reduction to bidiagonal form, then the routine of ssa_bidiag_ritz.  The
 * thick-restarted solver uses it for its projected matrix (an arrow block
 * followed by a bidiagonal one).  Errors: SSA_EINVAL.
 */
int ssa_dense_ritz(const double* A, int nr, int nc, int k, double* omega, double* P, double* Q);

/*
 * Profiling.  Kernel classes of the hot path, for ssa_profile_read:
 *   PASS1/PASS2/PASS3: the three FFT passes of one product X v or X^T u
 *   (Algorithms 2/3); DOTS/REDUCE/UPDATE: the Gram-Schmidt projection,
 *   coefficient reduction and update (Sec. 3.2.2); RITZ: Ritz vectors;
 *   RECON1/2/3: the FFT passes of the grouped rank-1 Hankelization
 *   (Algorithm 4); EMBED: the spectrum of the series (Algorithm 2, steps 1-2);
 *   DGKS2: the launches of a DGKS second Gram-Schmidt pass over the whole grid
 *   (long vectors), which return at once unless the criterion fired on the
 *   device; their algorithmic bytes are counted as 0.  CHECK: the stopping test
 *   on B_j and the Ritz coefficients on the device (eqs. lbdiagm1/lbdiagm2).
 *   On the fused path (1D, no thick restart, max(L, K) <= 2^20)
 *   PASS1 also finishes the previous Lanczos vector (the Gram-Schmidt update)
 *   and PASS3 also forms the projection partial sums, so UPDATE and DOTS stay 0.
 */
enum ssa_prof_class {
    SSA_PROF_PASS1 = 0, SSA_PROF_PASS2, SSA_PROF_PASS3, SSA_PROF_DOTS, SSA_PROF_REDUCE,
    SSA_PROF_UPDATE, SSA_PROF_RITZ, SSA_PROF_RECON1, SSA_PROF_RECON2, SSA_PROF_RECON3,
    SSA_PROF_EMBED, SSA_PROF_DGKS2, SSA_PROF_CHECK, SSA_PROF_NCLASSES
};

/*
 * ssa_profile_enable -- class_mask != 0: from now on count the launches and
 * algorithmic bytes of every kernel class, and bracket each launch of the
 * classes whose bit (1u << class) is set with HIP events on the plan's stream
 * (two event records per timed launch); 0: stop.  Either way the counters are
 * cleared (the stream is synchronized first).  Errors: SSA_EINVAL.
 */
int ssa_profile_enable(ssa_plan plan, unsigned class_mask);

/*
 * ssa_profile_read -- synchronize the plan's stream and report, for kernel
 * class cls since the last ssa_profile_enable: the number of launches, the
 * summed event-measured duration in milliseconds (-1 if the class was not
 * timed; with ssa_profile_sample, the timed launches' mean times the count) and
 * the summed algorithmic HBM bytes (the bytes the method must move: vectors
 * read and written, spectra, basis columns).  Errors: SSA_EINVAL, SSA_EDEVICE.
 */
int ssa_profile_read(ssa_plan plan, int cls, long long* launches, double* ms, double* bytes);

/*
 * ssa_profile_sample -- bracket only one launch in `every` (>= 1; default 1) of
 * each timed class with events, from the next launch on; ssa_profile_read then
 * reports the mean of the timed launches times the number of launches.  Fewer
 * event records disturb the stream less.  Errors: SSA_EINVAL.
 */
int ssa_profile_sample(ssa_plan plan, int every);

/* ssa_status_str -- static text for a status code. */
const char* ssa_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* SSA_H */
