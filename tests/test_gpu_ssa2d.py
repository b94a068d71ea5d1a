"""2D-SSA on the GPU against the 2D oracle (explicit Hankel-with-Hankel-blocks matrix,
Jacobi SVD, direct 2D diagonal averaging), through the C ABI.

The product X v of a 2D plan runs the 1D FFT product of the row-major flattened array
with the input scattered and the output gathered at row pitch Ny; the reconstruction is the
flattened 1D convolution of u_i and v_i divided by cnt_x(i) cnt_y(j), with positions of
count <= 2048 summed directly.  Tolerances are those of ``tests/parity.py``; the product
bound is the FFT bound of the 1D tests with the flattened length.
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


def fro2d(F, Lx, Ly):
    """|X|_F of the 2D trajectory matrix: F[i, j] appears cnt_x(i) cnt_y(j) times."""
    Nx, Ny = F.shape
    Kx, Ky = Nx - Lx + 1, Ny - Ly + 1
    i, j = np.arange(Nx), np.arange(Ny)
    cx = np.minimum.reduce([i + 1, np.full(Nx, Lx), np.full(Nx, Kx), Nx - i])
    cy = np.minimum.reduce([j + 1, np.full(Ny, Ly), np.full(Ny, Ky), Ny - j])
    return float(np.sqrt(np.sum(np.outer(cx, cy) * F * F)))


@pytest.mark.parametrize("Nx,Ny,Lx,Ly", [(12, 15, 5, 7), (30, 20, 25, 4), (1, 300, 1, 120), (40, 9, 13, 9),
                                         (17, 64, 1, 30), (64, 33, 31, 1), (50, 60, 25, 30)])
def test_products_2d(ssa, Nx, Ny, Lx, Ly):
    """X v and X^T u of the 2D trajectory matrix against the explicit matrix."""
    say(f"2D products {Nx}x{Ny} window {Lx}x{Ly}")
    rng = np.random.default_rng(Nx * Ny + Lx)
    F = inputs.array2d(Nx, Ny, seed=Nx + Ny)
    X = oracle.trajectory_2d(F, Lx, Ly)
    plan = ssa.Plan2D(Nx, Ny, Lx, Ly, 1)
    plan.embed(torch.tensor(F, device="cuda"))
    v = rng.normal(size=X.shape[1])
    u = rng.normal(size=X.shape[0])
    y = plan.matvec(torch.tensor(v, dtype=torch.float32, device="cuda")).cpu().numpy()
    yt = plan.matvec(torch.tensor(u, dtype=torch.float32, device="cuda"), transpose=True).cpu().numpy()
    ref = X @ v.astype(np.float32).astype(np.float64)
    reft = X.T @ u.astype(np.float32).astype(np.float64)
    M = plan.desc.M
    tol = 10.0 * EPS32 * np.log2(2 * M) * np.abs(F).sum()
    e1, e2 = np.abs(y - ref).max(), np.abs(yt - reft).max()
    say(f"  err X v {e1:.2e} (bound {tol * np.linalg.norm(v):.2e}), X^T u {e2:.2e}")
    assert e1 <= tol * np.linalg.norm(v)
    assert e2 <= tol * np.linalg.norm(u)
    plan.close()


def check_2d(ssa, F, Lx, Ly, k, **kw):
    Nx, Ny = F.shape
    Lc, Kc = Lx * Ly, (Nx - Lx + 1) * (Ny - Ly + 1)
    kr = min(k + 4, min(Lc, Kc))
    sA, UA, VA = oracle.ssa2d_dense(F, Lx, Ly, kr)
    plan = ssa.Plan2D(Nx, Ny, Lx, Ly, k, **kw)
    s, U, V, info = plan.truncated_svd(torch.tensor(F, device="cuda"), k)
    sg = s.cpu().numpy()
    Ug = U.cpu().numpy().T.astype(np.float64)
    Vg = V.cpu().numpy().T.astype(np.float64)
    fro = fro2d(F, Lx, Ly)
    rep = parity.compare_svd(sg, Ug, Vg, sA, UA, VA, k, fro)
    groups = [c for c in parity.clusters(sA, k, fro) if max(c) < k and sA[c[0]] > 1e-6 * sA[0]]
    rg = plan.reconstruct(s, U, V, groups).cpu().numpy().reshape(len(groups), -1)
    ro = oracle.reconstruct_2d(Nx, Ny, Lx, Ly, sA[:k], UA[:, :k], VA[:, :k], groups).reshape(len(groups), -1)
    rep["recon_err"] = parity.compare_recon(rg.astype(np.float64), ro, np.abs(F).max())
    rep["steps"] = info.steps
    rep["converged"] = info.converged
    rep["thick_restarts"] = info.thick_restarts
    say(f"  {Nx}x{Ny} window {Lx}x{Ly} k={k}: {rep}")
    plan.close()
    return rep


@pytest.mark.parametrize("Nx,Ny,Lx,Ly,k", [(30, 40, 15, 20, 8), (36, 30, 24, 20, 6), (24, 60, 8, 30, 10),
                                           (1, 400, 1, 150, 6), (48, 20, 48, 7, 4)])
def test_svd_2d_against_dense_oracle(ssa, Nx, Ny, Lx, Ly, k):
    say(f"2D SVD {Nx}x{Ny} window {Lx}x{Ly} k={k}")
    rep = check_2d(ssa, inputs.array2d(Nx, Ny, seed=3 * Nx + Ny), Lx, Ly, k)
    assert rep["converged"] == 1


def test_svd_2d_separable_and_plane_wave(ssa):
    """A separable array (Kronecker-structured trajectory matrix) and an exact rank-2 plane
    wave (surplus triples at sigma = 0)."""
    say("2D separable / plane wave")
    i, j = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    rng = np.random.default_rng(4)
    F = np.outer(np.cos(0.3 * np.arange(30)) + 0.2 * rng.normal(size=30), np.sin(0.2 * np.arange(40)) + 1.0)
    check_2d(ssa, F, 12, 16, 6)
    P = np.cos(0.41 * i + 0.93 * j + 0.3)
    plan = ssa.Plan2D(30, 40, 12, 16, 4)
    s, U, V, info = plan.truncated_svd(torch.tensor(P, device="cuda"), 4)
    sg = s.cpu().numpy()
    sA, _, _ = oracle.ssa2d_dense(P, 12, 16, 4)
    say(f"  plane wave sigma {sg} oracle {sA}")
    parity.assert_sigma(sg[:2], sA[:2])
    assert np.all(sg[2:] <= 1e-5 * sg[0])


def test_svd_2d_thick_restart_and_one_sided(ssa):
    F = inputs.array2d(30, 40, seed=11)
    say("2D thick restart")
    rep = check_2d(ssa, F, 15, 20, 8, d_max=20, restart_keep=12, check_every=64)
    assert rep["converged"] == 1 and rep["thick_restarts"] >= 1
    say("2D one-sided")
    rep = check_2d(ssa, F, 15, 20, 8, reorth=1)
    assert rep["converged"] == 1
