"""Planted mistakes in a scratch copy of the oracle must fail its pins.

Each case copies ``oracle/ssa_oracle.c`` to a temporary directory, applies one
plausible slip (a wrong sign, an off-by-one count, a reversed operand, a
shifted index), compiles it with gcc and runs the pins that are meant to catch
it against the mutant.  The committed oracle is never modified.
"""
import contextlib
import ctypes
import os
import shutil
import subprocess

import pytest

import oracle
from tests import test_oracle as pins

MUTATIONS = {
    "jacobi_rotation_sign": (
        "ap[i] = cs * xp - sn * xq;", "ap[i] = cs * xp + sn * xq;",
        [lambda: pins.test_jacobi_svd_matches_lapack((12, 5))]),
    "hankelize_count_off_by_one": (
        "g[n] = s / (double)cnt;", "g[n] = s / (double)(cnt + 1);",
        [pins.test_hankelize_paper_weights]),
    "rank1_correlation_not_convolution": (
        "s += u[i] * v[j];", "s += u[i] * v[K - 1 - j];",
        [pins.test_rank1_hankelize_is_linear_convolution_over_counts]),
    "matvec_reversed_rows": (
        "out[i] = dot(f + i, v, K);", "out[i] = dot(f + (L - 1 - i), v, K);",
        [lambda: pins.test_direct_products_match_explicit(64, 32)]),
    "bidiagonal_wrong_beta": (
        "B[(long)(c + 1) * jj + c] = beta[c + 2];", "B[(long)(c + 1) * jj + c] = beta[c + 1];",
        [lambda: pins.test_tier_b_matches_tier_a(300, 150, 10)]),
    "sampled_rows_off_by_one": (
        "out[q] = dot(f + rows[q], x, len);", "out[q] = dot(f + rows[q] + 1, x, len - 1);",
        [lambda: pins.test_sampled_rows_match_explicit(64, 32)]),
    "hankelize_at_count_dropped_end": (
        "out[q] = sigma * acc / (double)(a1 - a0 + 1);", "out[q] = sigma * acc / (double)(a1 - a0);",
        [pins.test_hankelize_at_matches_explicit_antidiagonals]),
    "hmatrix_lagged_vectors_of_base": (
        "const double* X = f + j + m;", "const double* X = f + i + m;",
        [lambda: pins.test_hmatrix_matches_numpy(30, 12, 9, 5, [1, 3])]),
    "realization_variance_biased": (
        "var[n] = R > 1 ? v / (double)(R - 1) : 0.0;", "var[n] = R > 1 ? v / (double)R : 0.0;",
        [pins.test_realization_stats_match_numpy]),
    "trajectory_2d_window_reversed": (
        "X[(a * Ly + b) * ncol + c * Ky + d] = F[(a + c) * Ny + (b + d)];",
        "X[(a * Ly + b) * ncol + c * Ky + d] = F[(a + c) * Ny + (Ly - 1 - b + d)];",
        [lambda: pins.test_trajectory_2d_of_separable_array_is_kronecker(6, 9, 3, 4)]),
    "hankelize_2d_count_off_by_one": (
        "G[i * Ny + j] = s / (double)cnt;", "G[i * Ny + j] = s / (double)(cnt + 1);",
        [pins.test_hankelize_2d_of_kronecker_factorizes]),
    "reconstruct_2d_v_transposed": (
        "acc += sigma[q] * U[(a * Ly + b) * k + q] * V[(c * Ky + d) * k + q];",
        "acc += sigma[q] * U[(a * Ly + b) * k + q] * V[(d * Kx + c) * k + q];",
        [pins.test_reconstruct_2d_sums_back_to_the_array]),
    "trajectory_shifted": (
        "X[i * K + j] = f[i + j];", "X[i * K + j] = f[i + j + (i + j + 1 < N)];",
        [pins.test_trajectory_matches_library_hankel]),
}


@contextlib.contextmanager
def mutant(tmp_path, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ssa_oracle.c")).read()
    assert old in src, old
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(path), "-lm"],
                   check=True)
    saved = oracle._load()
    oracle._lib = oracle._bind(ctypes.CDLL(str(so)))
    try:
        yield
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new, checks = MUTATIONS[name]
    with mutant(tmp_path, old, new):
        for check in checks:
            with pytest.raises((AssertionError, ValueError)):
                check()
    # and the unmodified oracle passes the same pins
    for check in checks:
        check()
