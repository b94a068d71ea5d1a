"""ssa_matvec_static (no allocation, the library's static device array) against the
existing entry point ssa_embed + ssa_matvec on the same inputs, through the C ABI.

Both run the same kernels with the same FFT schedule, so the products must agree
bit for bit.  Two calls of the static entry point run back to back, the second with
a smaller series, before either is compared: the second must not depend on what the
first left in the shared array.  The smaller product is also checked against the
FP64 oracle (Algorithms 2/3 against the direct sums of Sec. 2.1).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_0911_4498_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ssa():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0911_4498_amd import ssa as mod
    mod.load()
    return mod


def plan_product(ssa, f, L, x, transpose):
    p = ssa.Plan(len(f), L, 1)
    try:
        p.embed(f)
        y = p.matvec(x, transpose=transpose)
        torch.cuda.synchronize()
        return y.cpu().numpy()
    finally:
        p.close()


@pytest.mark.parametrize("transpose", [False, True])
def test_static_product_matches_plan_product(ssa, transpose):
    dev = torch.device("cuda:0")
    cases = [(100000, 50000, 11), (4001, 1300, 12)]  # the second call is smaller
    data = []
    for N, L, seed in cases:
        f = inputs.c2_series(N) if N == 100000 else inputs.c1_series(N)
        K = N - L + 1
        rng = np.random.default_rng(seed)
        x = rng.standard_normal(L if transpose else K).astype(np.float32)
        data.append((f, L, x))
    outs = []
    for f, L, x in data:
        say(f"static product: N={len(f)} L={L} transpose={transpose}")
        ft = torch.tensor(f, device=dev)
        y = ssa.matvec_static(ft, L, torch.tensor(x, device=dev), transpose=transpose)
        outs.append(y)
    torch.cuda.synchronize()
    for (f, L, x), y in zip(data, outs):
        got = y.cpu().numpy()
        ref = plan_product(ssa, f, L, x, transpose)
        say(f"  N={len(f)}: max |static - plan| = {np.abs(got - ref).max():.3e}")
        assert got.shape == ref.shape
        assert np.array_equal(got, ref)
    # the smaller case against the FP64 direct sums
    f, L, x = data[1]
    exact = oracle.rmatvec(f, L, x.astype(np.float64)) if transpose else oracle.matvec(f, L, x.astype(np.float64))
    got = outs[1].cpu().numpy().astype(np.float64)
    N = len(f)
    M = 2 * ((N + 1) // 2)
    bound = 10 * 2.0 ** -24 * np.log2(2 * M) * np.abs(f).sum() * np.linalg.norm(x)
    err = np.abs(got - exact).max()
    say(f"  N={N}: max |static - oracle| = {err:.3e} (bound {bound:.3e})")
    assert err <= bound
