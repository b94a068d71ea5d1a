"""The comparison rules of tests/parity.py, pinned on the CPU.

* rotation_factor is first-order perturbation theory for singular subspaces: for
  Gaussian perturbations of known size it must predict the exact rotation (FP64 SVD of
  the perturbed matrix) up to the sqrt(1/2) of averaging and the spread of a draw,
  both where a near-degenerate neighbour dominates and where the null space of a
  rectangular matrix does;
* fp32_model with FP64 arithmetic is Algorithm 1 with full reorthogonalization: it
  must reproduce the dense oracle's triples (so the model has no slip of its own);
* with float32 products it shows the FP32 limit: noise-floor clusters turn by more
  than 1e-4, and every cluster stays within half of angle_tolerance, which keeps
  1e-4 for the signal triples;
* residual bars: the FP32 model's triples meet half of RESID_REL with full
  reorthogonalization and half of RESID_REL_ONE_SIDED with one-sided, which does need
  the looser bar (its residuals pass RESID_REL).
"""
import numpy as np
import scipy.linalg

import oracle
from paper_0911_4498_amd import inputs
from tests import parity


def dense(f, L, k):
    s, U, V = oracle.ssa_dense(f, L, k)
    return s, U, V


def _orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _rotation_ratios(sig, rank, nr, nc, c, eta, draws=16, seed=0):
    """Exact rotation of cluster c of X = P diag(sig) Q^T under E ~ eta sigma_1 N(0, 1),
    divided by the first-order estimate eta G_c."""
    rng = np.random.default_rng(seed)
    P, Q = _orth(rng, nr, rank), _orth(rng, nc, rank)
    X = P @ np.diag(sig[:rank]) @ Q.T
    g = parity.rotation_factor(sig, c, nr, nc)
    out = []
    for _ in range(draws):
        E = eta * sig[0] * rng.standard_normal((nr, nc))
        Up, _, Vt = np.linalg.svd(X + E, full_matrices=False)
        out.append(max(parity.subspace_sin(P[:, c], Up[:, c]), parity.subspace_sin(Q[:, c], Vt[c].T)) / (eta * g))
    return np.array(out), g


def test_rotation_factor_near_degenerate_pair():
    # sigma_3 - sigma_4 = 3e-7: the pair's gap decides; rank 8 in 60 x 60 (the zeros are listed)
    sig = np.concatenate([[1.0, 0.5, 0.3, 0.3 - 3e-7, 0.1, 0.05, 0.02, 0.01], np.zeros(52)])
    r, g = _rotation_ratios(sig, 8, 60, 60, [2], 1e-10)
    assert g > 1e6
    assert 0.15 <= np.median(r) <= 1.5, r
    r, g = _rotation_ratios(sig, 8, 60, 60, [2, 3], 1e-10)  # merged: only the far gaps
    assert g < 100
    assert 0.3 <= np.median(r) <= 1.5, r


def test_rotation_factor_null_space_of_a_rectangular_matrix():
    # an isolated small sigma in a 6 x 300 matrix: the 294 extra directions decide
    sig = np.array([1.0, 0.6, 0.3, 0.1, 0.05, 0.01])
    for nr, nc in ((6, 300), (300, 6)):
        r, g = _rotation_ratios(sig, 6, nr, nc, [5], 1e-8)
        assert g > 1000
        assert 0.5 <= np.median(r) <= 1.5, r
    r, _ = _rotation_ratios(sig, 6, 6, 300, [0], 1e-8)
    assert 0.5 <= np.median(r) <= 1.5, r


def test_model_in_fp64_is_the_plain_algorithm():
    f = inputs.c1_series(600)
    L, k = 300, 10
    sA, UA, VA = dense(f, L, k + 4)
    s, U, V = parity.fp32_model(f, L, k + 4, dtype=np.float64)
    np.testing.assert_allclose(s[:k], sA[:k], rtol=1e-10)
    for c in parity.clusters(sA, k):
        if max(c) < k:
            assert parity.subspace_sin(UA[:, c], U[:, c]) < 1e-8
            assert parity.subspace_sin(VA[:, c], V[:, c]) < 1e-8


def test_model_in_fp64_window_longer_than_lag_count():
    f = inputs.c1_series(300)
    L, k = 200, 6
    sA, UA, VA = dense(f, L, k + 4)
    s, U, V = parity.fp32_model(f, L, k + 4, dtype=np.float64)
    assert U.shape[0] == L and V.shape[0] == 300 - L + 1
    np.testing.assert_allclose(s[:k], sA[:k], rtol=1e-10)
    for c in parity.clusters(sA, k):
        if max(c) < k:
            assert parity.subspace_sin(UA[:, c], U[:, c]) < 1e-8


def test_angle_tolerance_covers_the_fp32_model():
    cases = [(inputs.c1_series(1500), 750, 20), (inputs.c3_series(7, N=1600)[0], 400, 16),
             (inputs.c1_series(999), 333, 16)]
    beyond = 0
    for f, L, k in cases:
        sA, UA, VA = dense(f, L, k + 4)
        for seed in (1, 2):
            _, Um, Vm = parity.fp32_model(f, L, k + 4, seed=seed)
            for c in parity.clusters(sA, k):
                if max(c) >= k:
                    continue
                tol = parity.angle_tolerance(sA, c, UA.shape[0], VA.shape[0])
                sin = max(parity.subspace_sin(UA[:, c], Um[:, c]), parity.subspace_sin(VA[:, c], Vm[:, c]))
                assert sin <= tol / 2, (len(f), L, c, sin, tol)
                beyond += sin > parity.ANGLE_SIN
                if c[0] == 0:
                    assert tol == parity.ANGLE_SIN  # the leading triple keeps 1e-4
    assert beyond > 0  # the FP32 limit is real on these workloads


def test_residual_bars_cover_the_fp32_model():
    for f, L, k in ((inputs.c1_series(1000), 500, 10), (inputs.c1_series(1500), 750, 20)):
        X = scipy.linalg.hankel(f[:L], f[L - 1:])
        s, U, V = parity.fp32_model(f, L, k, d=64)
        assert parity.compare_residuals(X, s, U, V, k) <= parity.RESID_REL / 2
        s, U, V = parity.fp32_model(f, L, k, d=64, one_sided=True)
        worst = parity.compare_residuals(X, s, U, V, k, parity.RESID_REL_ONE_SIDED / 2)
        assert worst > parity.RESID_REL
