"""Seeded synthetic series shaped like the paper's workloads.

This module only draws input data (numpy PCG64, fixed draw order, t = 1..N);
it holds none of the SSA arithmetic.  It is the one piece shared by the
product's tests/benchmark and the oracle's tests.

Workloads (the paper's own data sets are not available; these stand in):

* ``c1``  -- N=1000, L=500, k=10: two sinusoids (periods 37 and 113), a linear
  trend 0.01 t and N(0, 0.1^2) noise.
* ``c2``  -- N=100000, L=50000, k=20: five sinusoids (periods log-uniform in
  [10, 2000], amplitudes U[0.5, 2], phases U[0, 2 pi]), an exp(-t/50000)
  trend and AR(1) noise (phi = 0.7, innovation sd 0.2, stationary start).
  Stands in for the long daily temperature record of Sec. 7.1
  (N = 86867, L = 43433).
* ``c3``  -- many independent series, N uniform in [2000, 20000],
  L = floor(N/2), k=16: two sinusoids (periods log-uniform in [10, 500],
  amplitudes U[0.5, 2.5]), trend (10/N) t, N(0, 0.1^2) noise.  Covers the
  N ~ 5000 birth-rate shape of Sec. 7.2.
* ``c4``  -- request stream: Poisson arrivals, N log-uniform in [1e3, 1e6],
  L in {N/4, N/2}, k uniform in [8, 32], c3 signal family.
* ``c5``  -- N = 2^24, L = N/2, k=50: eight sinusoids (periods log-uniform in
  [50, 1e6], amplitudes U[0.5, 2]), quadratic trend with U[-2, 2]
  coefficients in s = t/N, N(0, 0.5^2) noise.

Test signals with known structure (Sec. 6.3 finite-rank series and the
closed forms used as pins) are provided as well.
"""
from __future__ import annotations

import numpy as np

SEED_C1 = 1001
SEED_C2 = 1002
SEED_C3_BASE = 1003 * 10**6
SEED_C4_BASE = 1004 * 10**6
SEED_C5 = 1005


def _t(N: int) -> np.ndarray:
    return np.arange(1, N + 1, dtype=np.float64)


def c1_series(N: int = 1000, seed: int = SEED_C1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    t = _t(N)
    noise = rng.normal(0.0, 0.1, N)
    return (2.0 * np.sin(2 * np.pi * t / 37.0) + 1.5 * np.sin(2 * np.pi * t / 113.0 + 0.7)
            + 0.01 * t + noise)


def c2_series(N: int = 100_000, seed: int = SEED_C2) -> np.ndarray:
    rng = np.random.default_rng(seed)
    t = _t(N)
    periods = np.exp(rng.uniform(np.log(10.0), np.log(2000.0), 5))
    amps = rng.uniform(0.5, 2.0, 5)
    phases = rng.uniform(0.0, 2 * np.pi, 5)
    f = np.zeros(N)
    for P, A, ph in zip(periods, amps, phases):
        f += A * np.sin(2 * np.pi * t / P + ph)
    f += np.exp(-t / 50000.0)
    phi, sd = 0.7, 0.2
    z = rng.normal(0.0, 1.0, N)
    e = np.empty(N)
    e[0] = z[0] * sd / np.sqrt(1.0 - phi * phi)
    for i in range(1, N):
        e[i] = phi * e[i - 1] + sd * z[i]
    return f + e


def c3_shape(s: int, seed_base: int = SEED_C3_BASE):
    """(N, L) of batched series ``s`` (drawn first from the same stream as the series)."""
    rng = np.random.default_rng(seed_base + s)
    N = int(rng.integers(2000, 20001))
    return N, N // 2


def c3_series(s: int, seed_base: int = SEED_C3_BASE, N: int | None = None):
    """Series ``s`` of the batched workload: returns (f, N, L)."""
    rng = np.random.default_rng(seed_base + s)
    n_drawn = int(rng.integers(2000, 20001))
    if N is None:
        N = n_drawn
    L = N // 2
    return _two_sines_trend(rng, N), N, L


def _two_sines_trend(rng: np.random.Generator, N: int) -> np.ndarray:
    t = _t(N)
    periods = np.exp(rng.uniform(np.log(10.0), np.log(500.0), 2))
    amps = rng.uniform(0.5, 2.5, 2)
    phases = rng.uniform(0.0, 2 * np.pi, 2)
    f = np.zeros(N)
    for P, A, ph in zip(periods, amps, phases):
        f += A * np.sin(2 * np.pi * t / P + ph)
    f += (10.0 / N) * t
    f += rng.normal(0.0, 0.1, N)
    return f


def c4_request(r: int, seed_base: int = SEED_C4_BASE, n_max: int = 10**6):
    """Request ``r`` of the served stream: (f, N, L, k)."""
    rng = np.random.default_rng(seed_base + r)
    N = int(np.exp(rng.uniform(np.log(1e3), np.log(n_max))))
    L = N // 4 if rng.integers(0, 2) == 0 else N // 2
    k = int(rng.integers(8, 33))
    return _two_sines_trend(rng, N), N, L, k


def c4_arrivals(rate: float, n: int, seed: int = SEED_C4_BASE - 1) -> np.ndarray:
    """Poisson arrival times (seconds) of ``n`` requests at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def c5_series(N: int = 2**24, seed: int = SEED_C5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    periods = np.exp(rng.uniform(np.log(50.0), np.log(1e6), 8))
    amps = rng.uniform(0.5, 2.0, 8)
    phases = rng.uniform(0.0, 2 * np.pi, 8)
    c = rng.uniform(-2.0, 2.0, 3)
    t = _t(N)
    f = np.zeros(N)
    for P, A, ph in zip(periods, amps, phases):
        f += A * np.sin(2 * np.pi * t / P + ph)
    s = t / N
    f += c[0] + c[1] * s + c[2] * s * s
    f += rng.normal(0.0, 0.5, N)
    return f


def hmatrix_series(N: int = 400, Q: int = 200, seed: int = 1006) -> np.ndarray:
    """The structural-change example series: sin(2 pi n / 10) before n = Q, sin(2 pi n / 10.5)
    from n = Q on, plus 0.01 white noise (n = 1..N)."""
    rng = np.random.default_rng(seed)
    n = _t(N)
    f = np.where(n < Q, np.sin(2 * np.pi * n / 10.0), np.sin(2 * np.pi * n / 10.5))
    return f + 0.01 * rng.normal(0.0, 1.0, N)


# --- structured test signals -------------------------------------------------

def array2d(Nx: int, Ny: int, seed: int = 1007) -> np.ndarray:
    """2D-SSA input (Nx x Ny): three plane waves cos(2 pi (i / px + j / py) + phi) with periods
    log-uniform in [8, 200] along each axis and amplitudes U[0.5, 2], a smooth bilinear trend
    and N(0, 0.1^2) noise.  The paper has no 2D workload; this stands in for an image with a
    few periodic textures."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(Nx, dtype=np.float64), np.arange(Ny, dtype=np.float64), indexing="ij")
    F = np.zeros((Nx, Ny))
    for _ in range(3):
        px, py = np.exp(rng.uniform(np.log(8.0), np.log(200.0), 2))
        amp = rng.uniform(0.5, 2.0)
        phi = rng.uniform(0.0, 2 * np.pi)
        F += amp * np.cos(2 * np.pi * (i / px + j / py) + phi)
    c = rng.uniform(-1.0, 1.0, 3)
    F += c[0] + c[1] * i / Nx + c[2] * j / Ny
    F += rng.normal(0.0, 0.1, (Nx, Ny))
    return F


def sinusoid(N: int, period: float, amp: float = 1.0, phase: float = 0.0) -> np.ndarray:
    t = _t(N)
    return amp * np.cos(2 * np.pi * t / period + phase)


def geometric(N: int, a: float, rho: float) -> np.ndarray:
    return a * rho ** _t(N)


def rank5_example(N: int) -> np.ndarray:
    """Sec. 6.3's finite-rank series, read with n (not n/N) in the sine arguments."""
    n = _t(N)
    return (10.0 * np.exp(-5.0 * n / N) + np.sin(2 * np.pi * n / 13.0)
            + 2.5 * np.sin(2 * np.pi * n / 37.0))


def white(N: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, 1.0, N)


def start_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, 1.0, n)
