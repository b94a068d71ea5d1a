"""FP64 CPU oracle for Basic SSA -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never imports,
links or calls it, and it shares no code with the product.

The arithmetic lives in ``ssa_oracle.c`` (plain C, double precision); this
module only marshals numpy arrays through ctypes.  Each function cites the
part of the paper it follows:

* :func:`trajectory`        -- Sec. 2.1, the L-trajectory (Hankel) matrix.
* :func:`jacobi_svd`        -- Sec. 2.2, SVD by one-sided Jacobi rotations.
* :func:`ssa_dense`         -- Sec. 2.1-2.2, top-k triples of the explicit X
                               ("tier A": the definition written out).
* :func:`hankelize`         -- Sec. 2.4, diagonal averaging of any L x K matrix.
* :func:`rank1_hankelize`   -- Sec. 5, eq. for the rank-1 case as antidiagonal sums.
* :func:`reconstruct`       -- Sec. 2.3-2.4, grouping + diagonal averaging.
* :func:`matvec`/:func:`rmatvec` -- X v and X^T u evaluated row by row from the
                               series (X never stored), no FFT.
* :func:`lanczos_svd`       -- Sec. 3.1-3.2, Algorithm 1 with full
                               reorthogonalization ("tier B"), for sizes where
                               the explicit matrix does not fit.
* :func:`gkl_raw`           -- the raw Lanczos quantities, for the relations
                               of eqs. lbdiagm1 / lbdiagm2.
* :func:`trajectory_2d`, :func:`hankelize_2d`, :func:`ssa2d_dense`,
  :func:`reconstruct_2d`    -- 2D-SSA (the Hankel-with-Hankel-blocks case of
                               Sec. 1 and Sec. 3.3) from the definition.

Index convention: 0-based, ``X[i, j] = f[i + j]``, ``K = N - L + 1``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssa_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.c_long


def build(force: bool = True) -> str:
    """Compile ``ssa_oracle.c`` into ``liboracle.so`` next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_trajectory.argtypes = [_D, _L, _L, _D]
    lib.oracle_jacobi_svd.argtypes = [_D, _L, _L, ctypes.c_double, ctypes.c_int, _D, _D, _D]
    lib.oracle_hankelize.argtypes = [_D, _L, _L, _D]
    lib.oracle_rank1_hankelize.argtypes = [ctypes.c_double, _D, _L, _D, _L, _D]
    lib.oracle_reconstruct.argtypes = [_L, _L, ctypes.c_int, _D, _D, _D, _I, _I, ctypes.c_int, _D]
    lib.oracle_ssa_dense.argtypes = [_D, _L, _L, ctypes.c_int, _D, _D, _D]
    lib.oracle_matvec.argtypes = [_D, _L, _L, _D, _D]
    lib.oracle_rmatvec.argtypes = [_D, _L, _L, _D, _D]
    _LP = ctypes.POINTER(ctypes.c_long)
    lib.oracle_matvec_rows.argtypes = [_D, _L, _L, ctypes.c_int, _D, _LP, _L, _D]
    lib.oracle_hankelize_at.argtypes = [ctypes.c_double, _D, _L, _D, _L, _LP, _L, _D]
    lib.oracle_hmatrix.argtypes = [_D, _L, _L, _L, _L, _I, ctypes.c_int, _D]
    lib.oracle_realization_stats.argtypes = [_D, _L, _L, _L, ctypes.c_int, _D, _D, _D, _D]
    lib.oracle_lanczos_svd.argtypes = [_D, _L, _L, ctypes.c_int, ctypes.c_int, _D, _D,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       _D, _D, _D, _I]
    lib.oracle_gkl_raw.argtypes = [_D, _L, _L, ctypes.c_int, _D, _D, _D, _D, _D]
    lib.oracle_trajectory_2d.argtypes = [_D, _L, _L, _L, _L, _D]
    lib.oracle_hankelize_2d.argtypes = [_D, _L, _L, _L, _L, _D]
    lib.oracle_ssa2d_dense.argtypes = [_D, _L, _L, _L, _L, ctypes.c_int, _D, _D, _D]
    lib.oracle_reconstruct_2d.argtypes = [_L, _L, _L, _L, ctypes.c_int, _D, _D, _D, _I, _I, ctypes.c_int, _D]
    for name in ("oracle_trajectory", "oracle_jacobi_svd", "oracle_hankelize",
                 "oracle_rank1_hankelize", "oracle_reconstruct", "oracle_ssa_dense",
                 "oracle_matvec", "oracle_rmatvec", "oracle_lanczos_svd", "oracle_gkl_raw"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def trajectory(f, L: int) -> np.ndarray:
    """Sec. 2.1: the L x K trajectory matrix X[i, j] = f[i + j]."""
    f = _f64(f)
    N = f.size
    K = N - L + 1
    X = np.empty((L, K))
    rc = _load().oracle_trajectory(_dp(f), N, L, _dp(X))
    if rc < 0:
        raise ValueError("invalid N/L")
    return X


def jacobi_svd(A, tol: float = 1e-15, max_sweeps: int = 60):
    """Sec. 2.2: A = U diag(s) V^T by one-sided Jacobi; s descending, thin factors."""
    A = _f64(A)
    m, n = A.shape
    r = min(m, n)
    s = np.empty(r)
    U = np.empty((m, r))
    V = np.empty((n, r))
    sweeps = _load().oracle_jacobi_svd(_dp(A), m, n, tol, max_sweeps, _dp(s), _dp(U), _dp(V))
    if sweeps == -1:
        raise ValueError("bad shape")
    return s, U, V, sweeps


def ssa_dense(f, L: int, k: int):
    """Tier A (Sec. 2.1-2.2): the k leading triples of the explicit trajectory matrix."""
    f = _f64(f)
    N = f.size
    K = N - L + 1
    s = np.empty(k)
    U = np.empty((L, k))
    V = np.empty((K, k))
    rc = _load().oracle_ssa_dense(_dp(f), N, L, k, _dp(s), _dp(U), _dp(V))
    if rc < 0:
        raise ValueError("invalid arguments")
    return s, U, V


def hankelize(Y) -> np.ndarray:
    """Sec. 2.4: diagonal averaging of an arbitrary L x K matrix."""
    Y = _f64(Y)
    L, K = Y.shape
    g = np.empty(L + K - 1)
    _load().oracle_hankelize(_dp(Y), L, K, _dp(g))
    return g


def rank1_hankelize(sigma: float, u, v) -> np.ndarray:
    """Sec. 5: diagonal averaging of sigma * u v^T by direct antidiagonal sums."""
    u = _f64(u)
    v = _f64(v)
    g = np.empty(u.size + v.size - 1)
    _load().oracle_rank1_hankelize(float(sigma), _dp(u), u.size, _dp(v), v.size, _dp(g))
    return g


def reconstruct(N: int, L: int, sigma, U, V, groups) -> np.ndarray:
    """Sec. 2.3-2.4: one reconstructed series per group (list of triple indices)."""
    sigma = _f64(sigma)
    U = _f64(U)
    V = _f64(V)
    k = sigma.size
    offs = [0]
    mem: list[int] = []
    for g in groups:
        mem.extend(int(i) for i in g)
        offs.append(len(mem))
    offs_a = np.asarray(offs, dtype=np.int32)
    mem_a = np.asarray(mem if mem else [0], dtype=np.int32)
    out = np.empty((len(groups), N))
    rc = _load().oracle_reconstruct(N, L, k, _dp(sigma), _dp(U), _dp(V),
                                    offs_a.ctypes.data_as(_I), mem_a.ctypes.data_as(_I),
                                    len(groups), _dp(out))
    if rc < 0:
        raise ValueError("invalid arguments")
    return out


def matvec(f, L: int, v) -> np.ndarray:
    """X v, each entry a row of the trajectory matrix dotted with v."""
    f = _f64(f)
    v = _f64(v)
    out = np.empty(L)
    _load().oracle_matvec(_dp(f), f.size, L, _dp(v), _dp(out))
    return out


def rmatvec(f, L: int, u) -> np.ndarray:
    """X^T u, each entry a column of the trajectory matrix dotted with u."""
    f = _f64(f)
    u = _f64(u)
    out = np.empty(f.size - L + 1)
    _load().oracle_rmatvec(_dp(f), f.size, L, _dp(u), _dp(out))
    return out


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def matvec_rows(f, L: int, x, rows, transpose: bool = False) -> np.ndarray:
    """Selected entries of X x (rows of X) or of X^T x (columns), each a plain dot product."""
    f = _f64(f)
    x = _f64(x)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.size)
    rc = _load().oracle_matvec_rows(_dp(f), f.size, L, 1 if transpose else 0, _dp(x), _lp(rows), rows.size,
                                     _dp(out))
    if rc != 0:
        raise ValueError("invalid arguments")
    return out


def hankelize_at(sigma: float, u, v, pos) -> np.ndarray:
    """Sec. 2.4 at selected positions: mean of sigma u[a] v[b] over a + b = n, n in pos."""
    u = _f64(u)
    v = _f64(v)
    pos = np.ascontiguousarray(pos, dtype=np.int64)
    out = np.empty(pos.size)
    rc = _load().oracle_hankelize_at(float(sigma), _dp(u), u.size, _dp(v), v.size, _lp(pos), pos.size, _dp(out))
    if rc != 0:
        raise ValueError("invalid arguments")
    return out


def hmatrix(f, B: int, T: int, L: int, I) -> np.ndarray:
    """Structural-change detection: the H-matrix of heterogeneity indices g(base window i,
    test window j), base windows of length B, test windows of length T, window L, I 1-based."""
    f = _f64(f)
    N = f.size
    I = np.ascontiguousarray(I, dtype=np.int32)
    G = np.empty((N - B + 1, N - T + 1))
    rc = _load().oracle_hmatrix(_dp(f), N, B, T, L, I.ctypes.data_as(_I), I.size, _dp(G))
    if rc < 0:
        raise ValueError("invalid arguments")
    return G


def realization_stats(F, L: int, d: int, truth=None):
    """Repeated realizations: per point mean and (R-1)-normalized variance of the rank-d
    reconstructions of the rows of F, and their mean square error against truth."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    R, N = F.shape
    mean = np.empty(N)
    var = np.empty(N)
    mse = np.empty(N) if truth is not None else None
    tr = _f64(truth) if truth is not None else None
    rc = _load().oracle_realization_stats(_dp(F), R, N, L, d, _dp(tr) if tr is not None else None, _dp(mean),
                                          _dp(var), _dp(mse) if mse is not None else None)
    if rc < 0:
        raise ValueError("invalid arguments")
    return mean, var, mse


def lanczos_svd(f, L: int, k: int, p0, d_max: int | None = None, restart=None,
                check_every: int = 4, tol: float = 1e-13):
    """Tier B (Sec. 3.1-3.2): Algorithm 1 + full reorthogonalization, direct products.

    ``p0`` is the start vector (length L); ``restart`` an optional (n, max(L, K))
    array of replacement directions for vanishing alpha/beta.  Returns
    ``(sigma, U, V, steps, converged)``.
    """
    f = _f64(f)
    N = f.size
    K = N - L + 1
    if d_max is None:
        d_max = min(min(L, K), 10 * k + 40)
    p0 = _f64(p0)
    nmax = max(L, K)
    if restart is None:
        restart = np.zeros((0, nmax))
    restart = _f64(restart).reshape(-1, nmax)
    rs = restart if restart.size else np.zeros((1, nmax))
    s = np.empty(k)
    U = np.empty((L, k))
    V = np.empty((K, k))
    steps = ctypes.c_int(0)
    rc = _load().oracle_lanczos_svd(_dp(f), N, L, k, d_max, _dp(p0), _dp(rs),
                                    restart.shape[0], check_every, tol, _dp(s), _dp(U),
                                    _dp(V), ctypes.byref(steps))
    if rc < 0:
        raise ValueError("invalid arguments")
    return s, U, V, steps.value, rc == 0


def gkl_raw(f, L: int, d: int, p0):
    """d steps of Algorithm 1 (MGS-twice reorthogonalization): U (d+1, L), V (d+1, K),
    alpha[d+2], beta[d+2] (1-based indices as in the paper)."""
    f = _f64(f)
    N = f.size
    K = N - L + 1
    p0 = _f64(p0)
    Ub = np.zeros((d + 1, L))
    Vb = np.zeros((d + 1, K))
    a = np.zeros(d + 2)
    b = np.zeros(d + 2)
    rc = _load().oracle_gkl_raw(_dp(f), N, L, d, _dp(p0), _dp(Ub), _dp(Vb), _dp(a), _dp(b))
    if rc < 0:
        raise ValueError("invalid arguments")
    return Ub, Vb, a, b


def _groups_csr(groups):
    offs = [0]
    mem: list[int] = []
    for g in groups:
        mem.extend(int(i) for i in g)
        offs.append(len(mem))
    return np.asarray(offs, dtype=np.int32), np.asarray(mem if mem else [0], dtype=np.int32)


def trajectory_2d(F, Lx: int, Ly: int) -> np.ndarray:
    """2D-SSA trajectory matrix X[(a, b), (c, d)] = F[a + c, b + d]; rows a*Ly + b, columns c*Ky + d."""
    F = _f64(F)
    Nx, Ny = F.shape
    X = np.empty((Lx * Ly, (Nx - Lx + 1) * (Ny - Ly + 1)))
    if _load().oracle_trajectory_2d(_dp(F), Nx, Ny, Lx, Ly, _dp(X)) < 0:
        raise ValueError("invalid shape or window")
    return X


def hankelize_2d(Y, Nx: int, Ny: int, Lx: int, Ly: int) -> np.ndarray:
    """2D diagonal averaging of an (Lx Ly) x (Kx Ky) matrix into an Nx x Ny array."""
    Y = _f64(Y)
    G = np.empty((Nx, Ny))
    if _load().oracle_hankelize_2d(_dp(Y), Nx, Ny, Lx, Ly, _dp(G)) < 0:
        raise ValueError("invalid shape or window")
    return G


def ssa2d_dense(F, Lx: int, Ly: int, k: int):
    """2D-SSA from the definition: the k leading triples of the explicit 2D trajectory matrix."""
    F = _f64(F)
    Nx, Ny = F.shape
    L, K = Lx * Ly, (Nx - Lx + 1) * (Ny - Ly + 1)
    s = np.empty(k)
    U = np.empty((L, k))
    V = np.empty((K, k))
    if _load().oracle_ssa2d_dense(_dp(F), Nx, Ny, Lx, Ly, k, _dp(s), _dp(U), _dp(V)) < 0:
        raise ValueError("invalid arguments")
    return s, U, V


def reconstruct_2d(Nx: int, Ny: int, Lx: int, Ly: int, sigma, U, V, groups) -> np.ndarray:
    """2D grouping + diagonal averaging: one Nx x Ny array per group of triple indices."""
    sigma = _f64(sigma)
    U = _f64(U)
    V = _f64(V)
    offs, mem = _groups_csr(groups)
    out = np.empty((len(groups), Nx, Ny))
    rc = _load().oracle_reconstruct_2d(Nx, Ny, Lx, Ly, sigma.size, _dp(sigma), _dp(U), _dp(V),
                                       offs.ctypes.data_as(_I), mem.ctypes.data_as(_I), len(groups), _dp(out))
    if rc < 0:
        raise ValueError("invalid arguments")
    return out
