"""Host-side checks of the HIP library that need no GPU.

* the shared library loads and exports every function ``include/ssa.h`` declares;
* plan sizing (FFT length, split, workspace) and argument validation;
* the small bidiagonal solver used for the stopping test and the Ritz vectors,
  against LAPACK (numpy) on the explicit (d+1) x d bidiagonal.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0911_4498_amd import ssa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _built():
    if not os.path.exists(ssa.LIB_PATH):
        from paper_0911_4498_amd import build
        build.build()
    return ssa.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "ssa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(ssa_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    lib = _built()
    names = header_functions()
    assert "ssa_truncated_svd" in names and "ssa_reconstruct" in names and "ssa_embed_plan" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ssa.EXPORTED)


def make_plan(N, L, k, d_max=0):
    lib = _built()
    opts = ssa.SsaOpts(d_max, 0, 0.0, 0)
    ws = ctypes.c_size_t(0)
    h = ctypes.c_void_p()
    rc = lib.ssa_embed_plan(N, L, k, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
    return rc, h, ws.value


def describe(h):
    d = ssa.SsaPlanDesc()
    assert _built().ssa_plan_describe(h, ctypes.byref(d)) == 0
    return d


def smooth7(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("N,L,k", [(3, 2, 1), (1000, 500, 10), (100000, 50000, 20), (10007, 2501, 16),
                                   (999, 700, 5), (2**24, 2**23, 50), (65, 2, 2)])
def test_plan_sizes(N, L, k):
    lib = _built()
    rc, h, ws = make_plan(N, L, k)
    assert rc == 0
    d = describe(h)
    try:
        assert d.M >= N and d.M % 2 == 0
        assert d.M1 * d.M2 * 2 == d.M
        assert d.M1 <= 4096 and d.M2 <= 4096 and smooth7(d.M1) and smooth7(d.M2)
        assert d.K == N - L + 1
        r = min(L, N - L + 1)
        assert k <= d.d_max <= r
        assert ws == d.workspace_bytes and ws > 0
        # the smallest admissible M: no smaller even M >= N has an admissible split
        assert d.M // 2 - (N + 1) // 2 < 200
    finally:
        lib.ssa_plan_destroy(h)


@pytest.mark.parametrize("N,L,k", [(2, 1, 1), (10, 1, 1), (10, 10, 1), (10, 11, 1), (10, 5, 0),
                                   (10, 5, 6), (10, 8, 4), (-5, 2, 1)])
def test_plan_rejects_invalid(N, L, k):
    rc, h, _ = make_plan(N, L, k)
    assert rc == ssa.SSA_EINVAL
    assert not h.value


def test_unbound_plan_calls_fail_cleanly():
    lib = _built()
    rc, h, _ = make_plan(100, 40, 4)
    assert rc == 0
    try:
        assert lib.ssa_embed(h, ctypes.c_void_p(8)) == ssa.SSA_ENOMEM
        assert lib.ssa_matvec(h, 0, ctypes.c_void_p(8), ctypes.c_void_p(8)) == ssa.SSA_ENOMEM
        assert lib.ssa_plan_bind(h, None, 0, None) == ssa.SSA_EINVAL
        assert lib.ssa_plan_bind(h, ctypes.c_void_p(256), 16, None) == ssa.SSA_ENOMEM
        assert lib.ssa_plan_bind(h, ctypes.c_void_p(257), 1 << 40, None) == ssa.SSA_EINVAL
        info = ssa.SsaInfo()
        p8 = ctypes.c_void_p(256)
        assert lib.ssa_truncated_svd(h, p8, 100, 40, 5, p8, p8, p8, ctypes.byref(info)) == ssa.SSA_EINVAL
        assert lib.ssa_truncated_svd(h, p8, 101, 40, 2, p8, p8, p8, ctypes.byref(info)) == ssa.SSA_EMISMATCH
        assert lib.ssa_truncated_svd(h, p8, 100, 40, 2, p8, p8, p8, ctypes.byref(info)) == ssa.SSA_ENOMEM
    finally:
        lib.ssa_plan_destroy(h)
    assert ssa.status_str(ssa.SSA_ENONFINITE) == "series holds NaN or Inf"


def test_status_codes_and_info_layout():
    """The warning codes of ssa_truncated_svd and the report struct: the Python
    mirror of ssa_info must match the header's field order, including the status
    field that repeats the call's return value."""
    _built()
    assert ssa.SSA_WARN_NOT_CONVERGED == 1 and ssa.SSA_WARN_BREAKDOWN == 2
    assert "breakdown" in ssa.status_str(ssa.SSA_WARN_BREAKDOWN)
    assert "Krylov" in ssa.status_str(ssa.SSA_WARN_NOT_CONVERGED)
    text = open(os.path.join(ROOT, "include", "ssa.h")).read()
    body = text[text.index("typedef struct {\n    int steps;"):text.index("} ssa_info;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(\w+)(?:\[\d+\])?;", body)
    assert names == [f[0] for f in ssa.SsaInfo._fields_], names
    assert re.search(r"SSA_WARN_BREAKDOWN\s*=\s*2", text)


def test_matvec_static_host_checks():
    """ssa_matvec_static rejects bad arguments and series beyond its static array (N > 2^20)
    before it touches the device."""
    lib = _built()
    p8 = ctypes.c_void_p(256)
    assert lib.ssa_matvec_static(None, 100, 40, 0, p8, p8, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, 100, 40, 0, None, p8, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, 100, 40, 0, p8, None, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, 2, 1, 0, p8, p8, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, 100, 100, 1, p8, p8, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, 100, 1, 1, p8, p8, None) == ssa.SSA_EINVAL
    assert lib.ssa_matvec_static(p8, (1 << 20) + 1, 1000, 0, p8, p8, None) == ssa.SSA_ENOMEM


def test_fft_schedule_override():
    """ssa_opts.fft_m1 / fft_cb select the split of M' = M1*M2 and the columns per workgroup;
    invalid overrides are rejected."""
    lib = _built()

    def plan(m1, cb):
        opts = ssa.SsaOpts(0, 0, 0.0, 0, m1, cb)
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        rc = lib.ssa_embed_plan(100000, 50000, 20, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
        d = ssa.SsaPlanDesc()
        if rc == 0:
            assert lib.ssa_plan_describe(h, ctypes.byref(d)) == 0
            lib.ssa_plan_destroy(h)
        return rc, d

    rc, d = plan(0, 0)
    assert rc == 0 and d.M1 * d.M2 == 50000
    rc, d = plan(400, 16)
    assert rc == 0 and (d.M1, d.M2) == (400, 125)
    assert plan(300, 0)[0] == ssa.SSA_EINVAL      # does not divide M' = 50000
    assert plan(10, 0)[0] == ssa.SSA_EINVAL       # M2 = 5000 > 4096
    assert plan(1000, 16)[0] == ssa.SSA_EINVAL    # 16 columns of 1000 points exceed 32 per thread
    assert plan(200, 65)[0] == ssa.SSA_EINVAL


def _plan_mp(N, L, mp, m1=0, cb=0):
    lib = _built()
    opts = ssa.SsaOpts(0, 0, 0.0, 0, m1, cb, 0, 0, mp)
    ws = ctypes.c_size_t(0)
    h = ctypes.c_void_p()
    rc = lib.ssa_embed_plan(N, L, 4, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
    d = ssa.SsaPlanDesc()
    if rc == 0:
        assert lib.ssa_plan_describe(h, ctypes.byref(d)) == 0
        lib.ssa_plan_destroy(h)
    return rc, d


def test_fft_length_override():
    """ssa_opts.fft_mp picks a longer transform (any M >= N is exact): it must be 7-smooth,
    at least the smallest admissible M' and split into factors <= 4096."""
    rc, d = _plan_mp(100000, 50000, 51200)
    assert rc == 0 and d.M == 102400 and d.M1 * d.M2 == 51200 and d.M1 <= d.M2
    rc, d = _plan_mp(100000, 50000, 51200, 256, 2)
    assert rc == 0 and (d.M1, d.M2, d.cb) == (256, 200, 2)
    rc, d = _plan_mp(1000, 500, 512)
    assert rc == 0 and d.M == 1024
    assert _plan_mp(100000, 50000, 49152)[0] == ssa.SSA_EINVAL   # M = 98304 < N
    assert _plan_mp(100000, 50000, 50001)[0] == ssa.SSA_EINVAL   # not 7-smooth
    assert _plan_mp(100000, 50000, 50000 * 11)[0] == ssa.SSA_EINVAL
    assert _plan_mp(1000, 500, 8192 * 4096)[0] == ssa.SSA_EINVAL  # no split into factors <= 4096
    assert _plan_mp(100000, 50000, 51200, 300)[0] == ssa.SSA_EINVAL  # 300 does not divide 51200


def test_tuner_host_checks():
    """ssa_tune_workspace covers every candidate plan; ssa_tune_fft validates its arguments
    and the workspace before it touches the device."""
    lib = _built()
    b = ctypes.c_size_t(0)
    assert lib.ssa_tune_workspace(100000, 50000, ctypes.byref(b)) == 0
    rc, h, ws_auto = make_plan(100000, 50000, 1, 2)
    lib.ssa_plan_destroy(h)
    assert rc == 0 and b.value >= ws_auto + 4 * 2 * 100001
    opts = ssa.SsaOpts(2, 0, 0.0, 0, 0, 0, 0, 0, 51200)  # a candidate length above the smallest
    ws = ctypes.c_size_t(0)
    h = ctypes.c_void_p()
    assert lib.ssa_embed_plan(100000, 50000, 1, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h)) == 0
    lib.ssa_plan_destroy(h)
    assert b.value >= ws.value + 4 * 2 * 100001
    assert lib.ssa_tune_workspace(100, 100, ctypes.byref(b)) == ssa.SSA_EINVAL
    assert lib.ssa_tune_workspace(2, 1, ctypes.byref(b)) == ssa.SSA_EINVAL
    assert lib.ssa_tune_workspace(100, 40, None) == ssa.SSA_EINVAL
    best = ssa.SsaOpts()
    fake = ctypes.c_void_p(1 << 20)
    args = (1000, 500, fake, fake)
    need = ctypes.c_size_t(0)
    assert lib.ssa_tune_workspace(1000, 500, ctypes.byref(need)) == 0
    n = ctypes.c_int(0)
    assert lib.ssa_tune_fft(*args, need.value - 1, None, 5, ctypes.byref(best), None, 0, None, None,
                            ctypes.byref(n)) == ssa.SSA_ENOMEM
    assert lib.ssa_tune_fft(1000, 500, fake, ctypes.c_void_p((1 << 20) + 4), need.value, None, 5,
                            ctypes.byref(best), None, 0, None, None, None) == ssa.SSA_ENOMEM  # misaligned
    assert lib.ssa_tune_fft(*args, need.value, None, 0, ctypes.byref(best), None, 0, None, None,
                            None) == ssa.SSA_EINVAL  # reps
    assert lib.ssa_tune_fft(*args, need.value, None, 5, None, None, 0, None, None, None) == ssa.SSA_EINVAL
    assert lib.ssa_tune_fft(*args, need.value, None, 5, ctypes.byref(best), None, 4, None, None,
                            None) == ssa.SSA_EINVAL  # rows missing
    assert lib.ssa_tune_fft(1000, 500, None, fake, need.value, None, 5, ctypes.byref(best), None, 0, None, None,
                            None) == ssa.SSA_EINVAL
    assert (best.fft_mp, best.fft_m1, best.fft_cb) == (0, 0, 0)  # untouched on error


def test_schedule_table(tmp_path):
    """The tuner table: store/lookup round trip, and every stored entry is a valid schedule
    for its (N, L)."""
    from paper_0911_4498_amd import autotune
    path = str(tmp_path / "t.json")
    assert autotune.lookup(1000, 500, path) is None
    autotune.store(1000, 500, {"fft_mp": 512, "fft_m1": 16, "fft_cb": 2, "us_per_pair": 1.0}, path)
    autotune.store(100000, 50000, {"fft_mp": 51200, "fft_m1": 200, "fft_cb": 1}, path)
    assert autotune.lookup(1000, 500, path) == {"fft_mp": 512, "fft_m1": 16, "fft_cb": 2}
    assert autotune.lookup(1000, 501, path) is None
    assert list(autotune.load_table(path)) == ["1000:500", "100000:50000"]
    with open(path, "w") as fh:
        fh.write("[1, 2]")
    with pytest.raises(ValueError):
        autotune.load_table(path)
    for key, e in autotune.load_table(autotune.TABLE).items():
        N, L = (int(x) for x in key.split(":"))
        rc, d = _plan_mp(N, L, e["fft_mp"], e["fft_m1"], e["fft_cb"])
        assert rc == 0, key
        assert (d.M // 2, d.M1, d.cb) == (e["fft_mp"], e["fft_m1"], e["fft_cb"])
        assert e["us_per_pair"] <= e["auto"]["us_per_pair"]


def test_batch_validation_and_workspace():
    """The many-series entry points validate on the host before anything is enqueued, and
    the workspace a solve needs is a pure function of the series shapes."""
    lib = _built()
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t(0)
    assert lib.ssa_batch_plan(1000, 8, 4, None, ctypes.byref(ws), ctypes.byref(h)) == 0
    try:
        p = ctypes.c_void_p(256)
        offs = (ctypes.c_longlong * 3)(0, 100, 300)
        Ls = (ctypes.c_int * 2)(50, 150)  # the second window is longer than its lag count
        ks = (ctypes.c_int * 2)(4, 8)
        need = ctypes.c_size_t(0)
        assert lib.ssa_batch_workspace(h, 2, offs, Ls, ks, ctypes.byref(need)) == 0
        assert 0 < need.value <= ws.value
        one = ctypes.c_size_t(0)
        assert lib.ssa_batch_workspace(h, 1, offs, Ls, ks, ctypes.byref(one)) == 0
        assert one.value < need.value
        # unbound: valid arguments report the missing workspace, invalid ones EINVAL
        assert lib.ssa_batch_solve(h, 2, p, offs, Ls, ks, None, p, p, p, None, None) == ssa.SSA_ENOMEM
        bad_k = (ctypes.c_int * 2)(4, 9)  # above k_max
        assert lib.ssa_batch_solve(h, 2, p, offs, Ls, bad_k, None, p, p, p, None, None) == ssa.SSA_EINVAL
        bad_L = (ctypes.c_int * 2)(50, 200)  # L >= N
        assert lib.ssa_batch_solve(h, 2, p, offs, bad_L, ks, None, p, p, p, None, None) == ssa.SSA_EINVAL
        assert lib.ssa_batch_solve(h, 5, p, offs, Ls, ks, None, p, p, p, None, None) == ssa.SSA_EINVAL
        big = (ctypes.c_longlong * 2)(0, 1001)  # longer than n_max
        assert lib.ssa_batch_workspace(h, 1, big, Ls, ks, ctypes.byref(need)) == ssa.SSA_EINVAL
    finally:
        lib.ssa_batch_destroy(h)
    assert lib.ssa_batch_plan(20481, 8, 4, None, ctypes.byref(ws), ctypes.byref(h)) == ssa.SSA_EINVAL
    assert lib.ssa_batch_plan(1000, 33, 4, None, ctypes.byref(ws), ctypes.byref(h)) == ssa.SSA_EINVAL


def bidiag(alpha, beta, d):
    B = np.zeros((d + 1, d))
    for c in range(d):
        B[c, c] = alpha[c + 1]
        B[c + 1, c] = beta[c + 2]
    return B


@pytest.mark.parametrize("d,k,seed", [(5, 3, 0), (40, 10, 1), (120, 20, 2), (300, 50, 3), (1, 1, 4)])
def test_bidiag_ritz_matches_lapack(d, k, seed):
    rng = np.random.default_rng(seed)
    alpha = np.abs(rng.normal(size=d + 3)) + 0.1
    beta = np.abs(rng.normal(size=d + 3)) + 0.1
    alpha[0] = beta[0] = beta[1] = 0.0
    B = bidiag(alpha, beta, d)
    P_ref, s_ref, Qt_ref = np.linalg.svd(B, full_matrices=False)
    om, res = ssa.bidiag_ritz(alpha, beta, d, k)
    kk = min(k, d)
    np.testing.assert_allclose(om[:kk], s_ref[:kk], rtol=1e-12, atol=1e-13 * s_ref[0])
    np.testing.assert_allclose(res[:kk], alpha[d + 1] * np.abs(P_ref[d, :kk]), rtol=1e-7,
                               atol=1e-12 * s_ref[0])
    om2, _, P, Q = ssa.bidiag_ritz(alpha, beta, d, k, vectors=True)
    np.testing.assert_allclose(om2[:kk], s_ref[:kk], rtol=1e-12)
    # singular pairs: B q = omega p, orthonormal columns
    np.testing.assert_allclose(B @ Q[:, :kk], P[:, :kk] * om2[:kk], atol=1e-11 * s_ref[0])
    np.testing.assert_allclose(Q[:, :kk].T @ Q[:, :kk], np.eye(kk), atol=1e-11)
    np.testing.assert_allclose(P[:, :kk].T @ P[:, :kk], np.eye(kk), atol=1e-11)


def lanczos_bidiag(f, L, d, seed=1):
    """alpha, beta of d steps of Golub-Kahan-Lanczos in FP64 with full reorthogonalization
    on the explicit trajectory matrix (a test fixture, not the oracle)."""
    import scipy.linalg
    X = scipy.linalg.hankel(f[:L], f[L - 1:])
    Lh, K = X.shape
    U = np.zeros((Lh, d + 2))
    V = np.zeros((K, d + 1))
    al = np.zeros(d + 3)
    be = np.zeros(d + 3)
    p = np.random.default_rng(seed).normal(size=Lh)
    be[1] = np.linalg.norm(p)
    U[:, 0] = p / be[1]
    for j in range(1, d + 2):
        r = X.T @ U[:, j - 1] - (be[j] * V[:, j - 2] if j >= 2 else 0.0)
        for _ in range(2):
            r -= V[:, :j - 1] @ (V[:, :j - 1].T @ r)
        al[j] = np.linalg.norm(r)
        if j == d + 1:
            break
        V[:, j - 1] = r / al[j]
        q = X @ V[:, j - 1] - al[j] * U[:, j - 1]
        for _ in range(2):
            q -= U[:, :j] @ (U[:, :j].T @ q)
        be[j + 1] = np.linalg.norm(q)
        U[:, j] = q / be[j + 1]
    return al, be


@pytest.mark.parametrize("kind,d", [("c1", 80), ("c1", 120), ("white", 100), ("sine", 60)])
def test_stopping_test_on_lanczos_bidiagonals(kind, d):
    """The stopping test for d >= 48 (bisection and twisted factorizations) on bidiagonals
    from real Lanczos runs, where converged triples have eigenvector tails near 1e-20:
    Ritz values and residual bounds alpha_{d+1} |p_i[d]| against LAPACK."""
    from paper_0911_4498_amd import inputs
    if kind == "c1":
        f, L = inputs.c1_series(1000), 500
    elif kind == "white":
        f, L = inputs.white(800, 3), 400
    else:
        f, L = inputs.sinusoid(600, 23.0, 2.0) + 0.001 * inputs.white(600, 5), 300
    al, be = lanczos_bidiag(f, L, d)
    k = 16
    B = bidiag(al, be, d)
    P, s_ref, _ = np.linalg.svd(B, full_matrices=False)
    om, res = ssa.bidiag_ritz(al, be, d, k)
    np.testing.assert_allclose(om, s_ref[:k], rtol=1e-8)
    ref = al[d + 1] * np.abs(P[d, :k])
    big = ref > 1e-10 * s_ref[0]
    np.testing.assert_allclose(res[big], ref[big], rtol=1e-4)
    assert np.all(np.abs(res[~big] - ref[~big]) <= 1e-10 * s_ref[0])


def test_bidiag_ritz_clustered_and_zero_entries():
    """Exactly repeated singular values and vanishing alpha/beta (a split B) still give
    orthonormal vectors that span the right subspaces."""
    d, k = 12, 8
    alpha = np.zeros(d + 3)
    beta = np.zeros(d + 3)
    alpha[1:d + 1] = 1.0
    beta[2:d + 2] = 0.0
    alpha[3] = 2.0
    alpha[7] = 2.0  # sigma = 2 twice, then ones
    beta[5] = 0.5
    B = bidiag(alpha, beta, d)
    s_ref = np.linalg.svd(B, compute_uv=False)
    om, _, P, Q = ssa.bidiag_ritz(alpha, beta, d, k, vectors=True)
    np.testing.assert_allclose(om, s_ref[:k], rtol=1e-12)
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(B @ Q, P * om, atol=1e-10)


def arrow(omega, rho, a, b):
    """Projected matrix of a restarted bidiagonalization: diag(omega) with rho as column m,
    then b on the diagonal and a on the superdiagonal of the bidiagonal tail."""
    m = len(omega)
    n = m + len(b)
    B = np.zeros((n, n))
    B[np.arange(m), np.arange(m)] = omega
    B[:m, m] = rho
    for t in range(len(b)):
        B[m + t, m + t] = b[t]
        if t + 1 < len(b):
            B[m + t, m + t + 1] = a[t]
    return B


@pytest.mark.parametrize("shape,k,seed", [((7, 5), 3, 0), ((41, 40), 10, 1), ((60, 60), 20, 2),
                                          ((130, 90), 30, 3), ((1, 1), 1, 4), ((9, 4), 6, 5)])
def test_dense_ritz_matches_lapack(shape, k, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=shape)
    s_ref = np.linalg.svd(A, compute_uv=False)
    om, P, Q = ssa.dense_ritz(A, k)
    kk = min(k, shape[1])
    np.testing.assert_allclose(om[:kk], s_ref[:kk], rtol=1e-10, atol=1e-12 * s_ref[0])
    assert np.all(om[kk:] == 0) and np.all(P[:, kk:] == 0) and np.all(Q[:, kk:] == 0)
    np.testing.assert_allclose(A @ Q[:, :kk], P[:, :kk] * om[:kk], atol=1e-10 * s_ref[0])
    np.testing.assert_allclose(A.T @ P[:, :kk], Q[:, :kk] * om[:kk], atol=1e-10 * s_ref[0])
    np.testing.assert_allclose(Q[:, :kk].T @ Q[:, :kk], np.eye(kk), atol=1e-10)
    np.testing.assert_allclose(P[:, :kk].T @ P[:, :kk], np.eye(kk), atol=1e-10)


def test_dense_ritz_on_restart_shapes():
    """The two projected matrices of the restarted solver: the first cycle's (d+1) x d
    bidiagonal (same triples as the bidiagonal routine) and the arrow form of later
    cycles, whose last left-vector row gives the residual bound."""
    rng = np.random.default_rng(7)
    d, k = 30, 12
    alpha = np.abs(rng.normal(size=d + 3)) + 0.1
    beta = np.abs(rng.normal(size=d + 3)) + 0.1
    alpha[0] = beta[0] = beta[1] = 0.0
    B = bidiag(alpha, beta, d)
    om, P, Q = ssa.dense_ritz(B, k)
    om_b, res_b, P_b, Q_b = ssa.bidiag_ritz(alpha, beta, d, k, vectors=True)
    np.testing.assert_allclose(om, om_b, rtol=1e-12)
    np.testing.assert_allclose(alpha[d + 1] * np.abs(P[d]), res_b, rtol=1e-7, atol=1e-13 * om[0])
    for i in range(k):  # vectors agree up to sign
        sgn = np.sign(Q[:, i] @ Q_b[:, i])
        np.testing.assert_allclose(sgn * Q[:, i], Q_b[:, i], atol=1e-9)
        np.testing.assert_allclose(sgn * P[:, i], P_b[:, i], atol=1e-9)
    m = 14
    Ba = arrow(np.sort(rng.uniform(1, 10, m))[::-1], rng.normal(size=m) * 1e-3,
               np.abs(rng.normal(size=20)), np.abs(rng.normal(size=21)))
    U_ref, s_ref, _ = np.linalg.svd(Ba)
    om, P, Q = ssa.dense_ritz(Ba, m)
    np.testing.assert_allclose(om, s_ref[:m], rtol=1e-11)
    np.testing.assert_allclose(np.abs(P[-1]), np.abs(U_ref[-1, :m]), atol=1e-11)
    np.testing.assert_allclose(Ba @ Q, P * om, atol=1e-11 * s_ref[0])


def test_restart_keep_validation():
    lib = _built()

    def rc_of(N, L, k, d_max, keep):
        opts = ssa.SsaOpts(d_max, 0, 0.0, 0, 0, 0, keep)
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        rc = lib.ssa_embed_plan(N, L, k, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
        if rc == 0:
            lib.ssa_plan_destroy(h)
        return rc, ws.value

    assert rc_of(10000, 5000, 10, 40, 16)[0] == 0
    assert rc_of(10000, 5000, 10, 40, 9)[0] == ssa.SSA_EINVAL       # keep < k_max
    assert rc_of(10000, 5000, 10, 40, 39)[0] == ssa.SSA_EINVAL      # keep + 2 > d_max
    assert rc_of(10000, 5000, 10, 600, 16)[0] == ssa.SSA_EINVAL     # basis cap above 512
    assert rc_of(100, 20, 5, 64, 80)[0] == 0                        # whole Krylov space fits
    # the rotation scratch (keep columns of the longer basis) is part of the workspace
    assert rc_of(10000, 5000, 10, 40, 17)[1] >= rc_of(10000, 5000, 10, 40, 16)[1] + 4 * 5000


def test_reorth_option_validation():
    lib = _built()

    def rc_of(keep, reorth):
        opts = ssa.SsaOpts(40, 0, 0.0, 0, 0, 0, keep, reorth)
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        rc = lib.ssa_embed_plan(10000, 5000, 10, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
        if rc == 0:
            lib.ssa_plan_destroy(h)
        return rc

    assert rc_of(0, 1) == 0
    assert rc_of(0, 2) == ssa.SSA_EINVAL
    assert rc_of(16, 1) == ssa.SSA_EINVAL  # one-sided bases cannot be restarted
    for keep, reorth in ((16, 0), (0, 3)):  # the batch engine has no restart
        opts = ssa.SsaOpts(0, 0, 0.0, 0, 0, 0, keep, reorth)
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        assert lib.ssa_batch_plan(2000, 8, 4, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h)) == ssa.SSA_EINVAL
    opts = ssa.SsaOpts(0, 0, 0.0, 0, 0, 0, 0, 1)
    ws = ctypes.c_size_t(0)
    h = ctypes.c_void_p()
    assert lib.ssa_batch_plan(2000, 8, 4, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h)) == 0
    lib.ssa_batch_destroy(h)


def test_hmatrix_workspace_validation():
    """The H-matrix entry point checks its window sizes and index set on the host."""
    lib = _built()
    need = ctypes.c_size_t(0)

    def ws(N, B, T, L, I):
        Ia = (ctypes.c_int * len(I))(*I)
        return lib.ssa_hmatrix_workspace(N, B, T, L, Ia, len(I), ctypes.byref(need))

    assert ws(400, 100, 100, 50, [1, 2]) == 0 and need.value > 0
    small = need.value
    assert ws(800, 200, 200, 100, [1, 2]) == 0 and need.value > small
    assert ws(400, 100, 100, 99, [1, 2]) == ssa.SSA_EINVAL   # L must be below B - 1
    assert ws(400, 100, 40, 50, [1, 2]) == ssa.SSA_EINVAL    # L must not exceed T
    assert ws(400, 100, 100, 50, [0]) == ssa.SSA_EINVAL      # 1-based indices
    assert ws(400, 100, 100, 50, [33]) == ssa.SSA_EINVAL     # at most 32 triples
    assert ws(400, 500, 100, 50, [1]) == ssa.SSA_EINVAL      # base window longer than the series


def test_realizations_workspace_validation():
    lib = _built()
    need = ctypes.c_size_t(0)
    assert lib.ssa_realizations_workspace(64, 1000, 500, 5, ctypes.byref(need)) == 0 and need.value > 0
    assert lib.ssa_realizations_workspace(64, 1000, 500, 0, ctypes.byref(need)) == ssa.SSA_EINVAL
    assert lib.ssa_realizations_workspace(64, 1000, 1000, 5, ctypes.byref(need)) == ssa.SSA_EINVAL
    assert lib.ssa_realizations_workspace(64, 30000, 500, 5, ctypes.byref(need)) == ssa.SSA_EINVAL
    assert lib.ssa_realizations_workspace(0, 1000, 500, 5, ctypes.byref(need)) == ssa.SSA_EINVAL


def test_plan_2d_sizes_and_validation():
    lib = _built()

    def plan2d(Nx, Ny, Lx, Ly, k):
        opts = ssa.SsaOpts()
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        rc = lib.ssa_embed_plan_2d(Nx, Ny, Lx, Ly, k, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(h))
        d = describe(h) if rc == 0 else None
        if rc == 0:
            lib.ssa_plan_destroy(h)
        return rc, d

    rc, d = plan2d(40, 50, 20, 25, 8)
    assert rc == 0 and d.N == 2000 and d.L == 500 and d.K == 21 * 26 and d.M >= 2000
    assert plan2d(1, 100, 1, 30, 5)[0] == 0        # one row: Basic SSA of the row
    assert plan2d(30, 7, 30, 1, 1)[0] == 0         # full-height window: Kx = 1
    for bad in ((40, 50, 0, 25, 8), (40, 50, 41, 25, 8), (40, 50, 20, 51, 8), (1, 1, 1, 1, 1),
                (40, 50, 40, 50, 1), (5, 5, 2, 2, 5), (40, 50, 20, 25, 0)):
        assert plan2d(*bad)[0] == ssa.SSA_EINVAL, bad
