"""The comparison rules of tests/parity.py, pinned on the CPU.

* fp32_model with FP64 arithmetic is Algorithm 1 with full reorthogonalization: it
  must reproduce the dense oracle's triples (so the model has no slip of its own);
* with float32 products it shows the FP32 limit it is there to measure: on a c1
  series with k = 20 the isolated noise-floor triple 14 (relative gap 1.6e-3)
  turns by more than the 1e-4 tolerance, while the signal triples stay far below;
* resolved_clusters merges exactly such clusters with a neighbour and leaves the
  resolved ones alone.
"""
import numpy as np

import oracle
from paper_0911_4498_amd import inputs
from tests import parity


def dense(f, L, k):
    s, U, V = oracle.ssa_dense(f, L, k)
    return s, U, V


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


def test_model_in_fp32_measures_the_noise_floor_limit():
    f = inputs.c1_series(1500)
    L, k = 750, 20
    sA, UA, VA = dense(f, L, k + 4)
    model = parity.fp32_model(f, L, k + 4)
    _, Um, Vm = model
    sin = {tuple(c): parity.subspace_sin(UA[:, c], Um[:, c]) for c in parity.clusters(sA, k) if max(c) < k}
    assert max(sin[(i,)] for i in range(6)) < 1e-6          # the signal triples
    assert 1e-4 < sin[(14,)] < 3e-4, sin[(14,)]              # relative gap 1.6e-3 to triple 15
    cl = parity.resolved_clusters(sA, UA, VA, k, model)
    assert [0] in cl and [1] in cl and [5] in cl            # resolved clusters untouched
    merged = [c for c in cl if 14 in c][0]
    assert len(merged) > 1
    for c in cl:  # every cluster kept for the 1e-4 check is reproduced by the model
        if max(c) < k:
            assert parity.subspace_sin(UA[:, c], Um[:, c]) <= parity.ANGLE_SIN / 2, c
