"""The FFT schedule tuner on the device (needs an MI355X).

``ssa_tune_fft`` times the candidate schedules of the products through the C ABI.  The
checks: the report is consistent (the automatic schedule comes first, every candidate is a
valid split of a 7-smooth length >= ceil(N/2), the winner is the fastest row), and a plan
with the winning schedule gives the oracle's products and the dense oracle's triples.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_0911_4498_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ssa():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0911_4498_amd import ssa as mod
    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def smooth7(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def mv_tol(f, x, M):
    """FP32 FFT product bound: c eps log2(M) |f|_1 |x|_2 with c = 10."""
    return 10.0 * EPS32 * np.log2(2 * M) * np.abs(f).sum() * np.linalg.norm(x) + 1e-30


@pytest.mark.parametrize("N,L", [(1000, 500), (100000, 50000), (4099, 1234)])
def test_tuner_report_and_winner(ssa, N, L):
    say(f"tuner N={N} L={L}")
    f = inputs.c2_series(N)
    best, us_best, table = ssa.tune_fft(N, L, torch.tensor(f, device="cuda"), reps=5)
    say(f"  best {best} {us_best:.2f} us/pair over {len(table)} candidates; automatic {table[0]}")
    auto = ssa.Plan(N, L, 1).desc
    assert table[0][:3] == (auto.M // 2, auto.M1, auto.cb)
    for mp, m1, cb, us in table:
        assert 2 * mp >= N and smooth7(mp) and mp % m1 == 0
        assert m1 <= 4096 and mp // m1 <= 4096 and cb * m1 <= 8192
        assert np.isfinite(us) and us > 0
    assert us_best == min(r[3] for r in table)
    assert (best["fft_mp"], best["fft_m1"], best["fft_cb"]) in [r[:3] for r in table]
    # the winner's products against the oracle
    plan = ssa.Plan(N, L, 1, **best)
    assert plan.desc.M == 2 * best["fft_mp"] and plan.desc.M1 == best["fft_m1"] and plan.desc.cb == best["fft_cb"]
    plan.embed(torch.tensor(f, device="cuda"))
    rng = np.random.default_rng(N)
    v = rng.normal(size=N - L + 1)
    u = rng.normal(size=L)
    y = plan.matvec(torch.tensor(v, dtype=torch.float32, device="cuda")).cpu().numpy()
    yt = plan.matvec(torch.tensor(u, dtype=torch.float32, device="cuda"), transpose=True).cpu().numpy()
    ref = oracle.matvec(f, L, v.astype(np.float32).astype(np.float64))
    reft = oracle.rmatvec(f, L, u.astype(np.float32).astype(np.float64))
    assert np.abs(y - ref).max() <= mv_tol(f, v, plan.desc.M)
    assert np.abs(yt - reft).max() <= mv_tol(f, u, plan.desc.M)
    plan.close()


def test_tuned_schedule_solve_matches_dense_oracle(ssa):
    """c1 (N=1000, L=500, k=10) with the tuner's schedule and with a longer transform than
    the smallest: triples and reconstructions within the parity tolerances."""
    say("tuned solve c1")
    f = inputs.c1_series()
    N, L, k = 1000, 500, 10
    best, _, _ = ssa.tune_fft(N, L, torch.tensor(f, device="cuda"), reps=3)
    sA, UA, VA = oracle.ssa_dense(f, L, k + 4)
    fro = parity.frobenius(f, L)
    for sched in (best, {"fft_mp": 640, "fft_m1": 20, "fft_cb": 2}):
        plan = ssa.Plan(N, L, k, **sched)
        s, U, V, info = plan.truncated_svd(torch.tensor(f, device="cuda"), k)
        rep = parity.compare_svd(s.cpu().numpy(), U.cpu().numpy().T.astype(np.float64),
                                 V.cpu().numpy().T.astype(np.float64), sA, UA, VA, k, fro)
        groups = [c for c in parity.clusters(sA, k, fro) if max(c) < k]
        rg = plan.reconstruct(s, U, V, groups).cpu().numpy()
        ro = oracle.reconstruct(N, L, sA[:k], UA[:, :k], VA[:, :k], groups)
        rep["recon_err"] = parity.compare_recon(rg, ro, np.abs(f).max())
        say(f"  schedule {sched}: {rep}")
        assert info.converged == 1
        plan.close()
