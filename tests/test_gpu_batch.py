"""The many-series path (lockstep launches, one workgroup per series) against the
FP64 oracle.

Each series of a batch is compared with the oracle exactly as the single-series
path is (``tests/parity.py``): sigma, vector subspaces per cluster, and the
elementary reconstructions (summed over a cluster).  A series must give the
same bits alone and inside a batch (same key).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_0911_4498_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ssa():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0911_4498_amd import ssa as mod
    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_one(f, L, k, sig, U, V, rec, dense=True):
    N = len(f)
    K = N - L + 1
    sg = sig.cpu().numpy()
    Ug = U.cpu().numpy().T.astype(np.float64)
    Vg = V.cpu().numpy().T.astype(np.float64)
    kr = min(k + 4, min(L, K))
    if dense:
        sA, UA, VA = oracle.ssa_dense(f, L, kr)
    else:
        p0 = inputs.start_vector(L, 7)
        sA, UA, VA, _, conv = oracle.lanczos_svd(f, L, kr, p0, tol=1e-12)
        assert conv
    cl = parity.clusters(sA, k)
    rep = parity.compare_svd(sg, Ug, Vg, sA, UA, VA, k, cl=cl)
    groups = [c for c in cl if max(c) < k and sA[c[0]] > 1e-6 * sA[0]]
    if groups:  # white noise can leave one cluster straddling k: then sigma and subspaces only
        rg = rec.cpu().numpy().astype(np.float64)
        ref = oracle.reconstruct(N, L, sA[:k], UA[:, :k], VA[:, :k], groups)
        got = np.array([rg[c].sum(axis=0) for c in groups])
        rep["recon_err"] = parity.compare_recon(got, ref, np.abs(f).max())
    return rep


def small_batch(n):
    rng = np.random.default_rng(2024)
    series, Ls, ks = [], [], []
    for s in range(n):
        N = int(rng.integers(60, 1500))
        kind = s % 4
        if kind == 0:
            f, _, _ = inputs.c3_series(s, N=N)
        elif kind == 1:
            f = inputs.c1_series(N)
        elif kind == 2:
            f = inputs.sinusoid(N, 17.0, 2.0) + 0.05 * inputs.white(N, s)
        else:
            f = inputs.white(N, s)
        L = N // 2 if s % 5 else (3 * N) // 4  # some windows longer than the lag count
        k = int(rng.integers(4, 17))
        series.append(f)
        Ls.append(L)
        ks.append(min(k, L, N - L + 1))
    return series, Ls, ks


def test_batch_small_series_match_oracle(ssa):
    series, Ls, ks = small_batch(12)
    say("batch of 12 series: solving")
    b = ssa.Batch(n_max=1500, k_max=16, max_series=64)
    out = b.solve(series, Ls, ks)
    info = out["info"].cpu().numpy()
    say("batch of 12 series: solved")
    for s, (f, L, k) in enumerate(zip(series, Ls, ks)):
        say(f"batch series {s}: N={len(f)} L={L} k={k} steps={info[s, 0]} conv={info[s, 1]}")
        rep = compare_one(f, L, k, out["sigma"][s], out["U"][s], out["V"][s], out["recon"][s])
        say(f"   {rep}")


def test_batch_one_sided_reorth_matches_oracle(ssa):
    """reorth=1: only the length-min(L,K) basis is reorthogonalized; same tolerances."""
    series, Ls, ks = small_batch(12)
    say("batch of 12 series, one-sided: solving")
    b = ssa.Batch(n_max=1500, k_max=16, max_series=64, reorth=1)
    out = b.solve(series, Ls, ks)
    info = out["info"].cpu().numpy()
    for s, (f, L, k) in enumerate(zip(series, Ls, ks)):
        say(f"batch one-sided series {s}: N={len(f)} L={L} k={k} steps={info[s, 0]} conv={info[s, 1]}")
        rep = compare_one(f, L, k, out["sigma"][s], out["U"][s], out["V"][s], out["recon"][s])
        say(f"   {rep}")
    f, N, L = inputs.c3_series(5, N=12000)
    say("c3 series 5, one-sided: solving")
    b2 = ssa.Batch(n_max=20480, k_max=16, max_series=4, reorth=1)
    out = b2.solve([f], [L], [16])
    rep = compare_one(f, L, 16, out["sigma"][0], out["U"][0], out["V"][0], out["recon"][0], dense=False)
    say(f"   {rep}")


def test_batch_alone_equals_in_the_mix(ssa):
    series, Ls, ks = small_batch(32)
    keys = [7000 + s for s in range(32)]
    b = ssa.Batch(n_max=1500, k_max=16, max_series=64)
    say("32 series mixed: solving")
    mixed = b.solve(series, Ls, ks, keys=keys)
    torch.cuda.synchronize()
    for s in (0, 5, 17, 31):
        say(f"series {s} alone: solving")
        alone = b.solve([series[s]], [Ls[s]], [ks[s]], keys=[keys[s]])
        torch.cuda.synchronize()
        for key in ("sigma", "U", "V", "recon"):
            a = alone[key][0].cpu().numpy()
            m = mixed[key][s].cpu().numpy()
            assert np.array_equal(a, m), (s, key)


@pytest.mark.parametrize("s", [3, 11])
def test_batch_c3_series_match_oracle(ssa, s):
    """Series of the many-series workload (N up to 20000, L = N/2, k = 16) against the
    tier-B oracle (direct products), one series in a batch of four."""
    f, N, L = inputs.c3_series(s)
    N = min(N, 12000)
    f, N, L = inputs.c3_series(s, N=N)
    others = [inputs.c3_series(t, N=2000)[0] for t in range(3)]
    b = ssa.Batch(n_max=20480, k_max=16, max_series=8)
    say(f"c3 series {s}: solving in a batch of four")
    out = b.solve([f] + others, [L] + [1000] * 3, [16] * 4)
    info = out["info"].cpu().numpy()
    say(f"c3 series {s}: N={N} steps={info[0, 0]} conv={info[0, 1]}")
    rep = compare_one(f, L, 16, out["sigma"][0], out["U"][0], out["V"][0], out["recon"][0], dense=False)
    say(f"   {rep}")


@pytest.mark.parametrize("N,L", [(20480, 10240), (20479, 5000)])
def test_batch_longest_series_match_oracle(ssa, N, L):
    """The longest series the batched engine holds (M' = 10240 points in LDS: every load
    batch of the product kernel in use), with L = N/2 and an odd N with L < K, against the
    tier-B oracle, in a batch with three short series."""
    f, _, _ = inputs.c3_series(7, N=N)
    others = [inputs.c3_series(t, N=900)[0] for t in range(3)]
    b = ssa.Batch(n_max=20480, k_max=16, max_series=8)
    say(f"longest series: N={N} L={L}: solving in a batch of four")
    out = b.solve([f] + others, [L] + [450] * 3, [8] * 4)
    info = out["info"].cpu().numpy()
    say(f"longest series: N={N} steps={info[0, 0]} conv={info[0, 1]}")
    rep = compare_one(f, L, 8, out["sigma"][0], out["U"][0], out["V"][0], out["recon"][0], dense=False)
    say(f"   {rep}")
    for s in range(1, 4):
        rep = compare_one(others[s - 1], 450, 8, out["sigma"][s], out["U"][s], out["V"][s], out["recon"][s])
        say(f"   short series {s}: {rep}")


def test_batch_full_many_series_workload(ssa):
    """The many-series workload exactly as the benchmark launches it: 4096 series (N uniform in
    [2000, 20000], L = N/2, k = 16) in one batch.  Three sampled series against the oracle
    (dense where N <= 4000, else tier B), residual and orthonormality certificates (FP64,
    numpy FFT) for 64 sampled series, and ordering / convergence for all of them."""
    ns, k = 4096, 16
    say(f"full many-series workload: generating {ns} series")
    host = [inputs.c3_series(s) for s in range(ns)]
    series = [torch.tensor(f, device="cuda") for f, _, _ in host]
    Ls = [L for _, _, L in host]
    b = ssa.Batch(n_max=20000, k_max=k, max_series=ns)
    say("full many-series workload: solving")
    out = b.solve(series, Ls, [k] * ns, keys=list(range(ns)))
    info = out["info"].cpu().numpy()
    say(f"  mean steps {info[:, 0].mean():.1f}, converged {info[:, 1].mean():.4f}")
    assert info[:, 1].mean() >= 0.99
    for s in range(ns):
        sg = out["sigma"][s].cpu().numpy()
        assert np.all(np.diff(sg) <= 1e-12 * sg[0]) and sg[-1] > 0, s
    rng = np.random.default_rng(4096)
    for s in sorted(rng.choice(ns, 3, replace=False)):
        f, N, L = host[s]
        say(f"  series {s}: N={N} oracle comparison")
        rep = compare_one(f, L, k, out["sigma"][s], out["U"][s], out["V"][s], out["recon"][s], dense=N <= 4000)
        say(f"     {rep}")
    worst = 0.0
    for s in sorted(rng.choice(ns, 64, replace=False)):
        f, N, L = host[s]
        K = N - L + 1
        sg = out["sigma"][s].cpu().numpy()
        U = out["U"][s].cpu().numpy().astype(np.float64)
        V = out["V"][s].cpu().numpy().astype(np.float64)
        M = 1 << int(np.ceil(np.log2(2 * N)))
        F = np.fft.rfft(f, M)
        for i in range(k):
            y = np.fft.irfft(F * np.fft.rfft(V[i][::-1], M), M)[K - 1:K - 1 + L]
            r1 = np.linalg.norm(y - sg[i] * U[i])
            y = np.fft.irfft(F * np.fft.rfft(U[i][::-1], M), M)[L - 1:L - 1 + K]
            r2 = np.linalg.norm(y - sg[i] * V[i])
            worst = max(worst, r1 / sg[0], r2 / sg[0])
        for B in (U, V):
            assert np.abs(B @ B.T - np.eye(k)).max() <= 1e-5, s
    say(f"  worst residual / sigma_1 over 64 sampled series: {worst:.2e}")
    assert worst <= 1e-5
