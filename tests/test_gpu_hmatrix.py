"""Structural-change detection on the GPU (ssa_hmatrix) against the FP64 oracle's
H-matrix, computed from the definition (eq. g)."""
import sys

import numpy as np
import pytest

import oracle
from paper_0911_4498_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# The eigenvectors come from the FP32 path (angles ~1e-6 against the oracle); an index is a
# ratio of FP64 sums of their squared projections, so its error is of the same order.
G_TOL = 2e-5


@pytest.fixture(scope="module")
def ssa():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0911_4498_amd import ssa as mod
    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_hmatrix_paper_example(ssa):
    """N = 400, Q = 200, B = T = 100, L = 50, I = {1, 2}."""
    f = inputs.hmatrix_series(400, 200, 5)
    say("H-matrix N=400 B=T=100 L=50 I={1,2}")
    G = ssa.hmatrix(f, 100, 100, 50, [1, 2]).cpu().numpy()
    ref = oracle.hmatrix(f, 100, 100, 50, [1, 2])
    err = np.abs(G - ref).max()
    say(f"  max |G - G_oracle| = {err:.2e}; G range [{G.min():.2e}, {G.max():.3f}]")
    assert err <= G_TOL
    assert G[0, -1] > 0.1 and G[0, 0] < 1e-3


@pytest.mark.parametrize("N,B,T,L,I", [(300, 80, 60, 30, [1, 2]), (257, 64, 64, 20, [3, 4]),
                                       (500, 120, 90, 40, [1, 2, 3, 4])])
def test_hmatrix_other_shapes(ssa, N, B, T, L, I):
    """Two sinusoids of different amplitude (two well separated pairs) with a period change
    in the middle; the index sets take whole pairs, so each span is unique."""
    t = np.arange(1, N + 1)
    f = 3.0 * np.sin(2 * np.pi * t / 12.0) + 1.2 * np.sin(2 * np.pi * t / np.where(t < N // 2, 29.0, 23.0))
    f = f + 0.01 * inputs.white(N, N)
    say(f"H-matrix N={N} B={B} T={T} L={L} I={I}")
    G = ssa.hmatrix(f, B, T, L, I).cpu().numpy()
    ref = oracle.hmatrix(f, B, T, L, I)
    err = np.abs(G - ref).max()
    say(f"  max |G - G_oracle| = {err:.2e}")
    assert err <= G_TOL
