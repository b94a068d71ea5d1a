"""ctypes binding of the HIP library (``include/ssa.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libssa_hip.so``.  PyTorch supplies device memory (the workspace
and the result tensors) and the stream.  There is no CPU fallback: if the
library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssa_hip.so")

SSA_OK = 0
SSA_WARN_NOT_CONVERGED = 1
SSA_WARN_BREAKDOWN = 2
SSA_EINVAL = -1
SSA_ENOMEM = -2
SSA_ENONFINITE = -3
SSA_EDEVICE = -4
SSA_EMISMATCH = -5
SSA_ESTATE = -6

_c_ll = ctypes.c_longlong
_c_p = ctypes.c_void_p


class SsaOpts(ctypes.Structure):
    _fields_ = [("d_max", ctypes.c_int), ("check_every", ctypes.c_int), ("tol", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("fft_m1", ctypes.c_int), ("fft_cb", ctypes.c_int),
                ("restart_keep", ctypes.c_int), ("reorth", ctypes.c_int), ("fft_mp", ctypes.c_longlong),
                ("unfused", ctypes.c_int)]


class SsaInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("converged", ctypes.c_int), ("restarts", ctypes.c_int),
                ("dgks_passes", ctypes.c_int), ("steps_run", ctypes.c_int), ("resid", ctypes.c_double * 64),
                ("thick_restarts", ctypes.c_int), ("status", ctypes.c_int), ("half_step_launches", ctypes.c_int)]


class SsaPlanDesc(ctypes.Structure):
    _fields_ = [("N", _c_ll), ("L", _c_ll), ("K", _c_ll), ("M", _c_ll), ("M1", _c_ll), ("M2", _c_ll),
                ("d_max", ctypes.c_int), ("k_max", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t),
                ("cb", ctypes.c_int)]


EXPORTED = ("ssa_embed_plan", "ssa_embed_plan_2d", "ssa_plan_bind", "ssa_embed", "ssa_matvec", "ssa_matvec_static",
            "ssa_truncated_svd",
            "ssa_reconstruct", "ssa_plan_describe", "ssa_plan_destroy", "ssa_status_str",
            "ssa_bidiag_ritz", "ssa_dense_ritz", "ssa_profile_enable", "ssa_profile_read", "ssa_profile_sample",
            "ssa_batch_plan", "ssa_batch_workspace", "ssa_batch_bind", "ssa_batch_solve",
            "ssa_batch_profile_enable", "ssa_batch_profile_read", "ssa_batch_destroy",
            "ssa_server_create", "ssa_server_enable_long", "ssa_server_create_stub", "ssa_server_request_bytes", "ssa_server_submit", "ssa_server_step",
            "ssa_server_status", "ssa_server_destroy", "ssa_hmatrix_workspace", "ssa_hmatrix",
            "ssa_realizations_workspace", "ssa_realizations", "ssa_tune_workspace", "ssa_tune_fft")

# kernel classes of ssa_batch_profile_read (enum ssa_batch_prof_class)
BATCH_PROF_CLASSES = ("init", "conv", "cgs", "check", "ritz", "hankel")

# kernel classes of ssa_profile_read (enum ssa_prof_class)
PROF_CLASSES = ("pass1", "pass2", "pass3", "cgs_dots", "cgs_reduce", "cgs_update", "ritz",
                "recon_pass1", "recon_pass2", "recon_pass3", "embed", "dgks2", "check")

_lib = None


class SsaError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_str(code)} ({code})")


def load():
    """Load ``libssa_hip.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_0911_4498_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ssa_embed_plan.argtypes = [_c_ll, _c_ll, ctypes.c_int, ctypes.POINTER(SsaOpts),
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_c_p)]
    lib.ssa_embed_plan_2d.argtypes = [_c_ll, _c_ll, _c_ll, _c_ll, ctypes.c_int, ctypes.POINTER(SsaOpts),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_c_p)]
    lib.ssa_plan_bind.argtypes = [_c_p, _c_p, ctypes.c_size_t, _c_p]
    lib.ssa_embed.argtypes = [_c_p, _c_p]
    lib.ssa_matvec.argtypes = [_c_p, ctypes.c_int, _c_p, _c_p]
    lib.ssa_matvec_static.argtypes = [_c_p, _c_ll, _c_ll, ctypes.c_int, _c_p, _c_p, _c_p]
    lib.ssa_truncated_svd.argtypes = [_c_p, _c_p, _c_ll, _c_ll, ctypes.c_int, _c_p, _c_p, _c_p,
                                      ctypes.POINTER(SsaInfo)]
    lib.ssa_reconstruct.argtypes = [_c_p, _c_p, _c_p, _c_p, ctypes.c_int, _c_p, _c_p, ctypes.c_int, _c_p]
    lib.ssa_plan_describe.argtypes = [_c_p, ctypes.POINTER(SsaPlanDesc)]
    lib.ssa_plan_destroy.argtypes = [_c_p]
    lib.ssa_plan_destroy.restype = None
    lib.ssa_status_str.argtypes = [ctypes.c_int]
    lib.ssa_status_str.restype = ctypes.c_char_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ssa_bidiag_ritz.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    lib.ssa_dense_ritz.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
    lib.ssa_profile_enable.argtypes = [_c_p, ctypes.c_uint]
    lib.ssa_profile_read.argtypes = [_c_p, ctypes.c_int, ctypes.POINTER(_c_ll), dp, dp]
    lib.ssa_profile_sample.argtypes = [_c_p, ctypes.c_int]
    lib.ssa_batch_plan.argtypes = [_c_ll, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SsaOpts),
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_c_p)]
    lib.ssa_batch_workspace.argtypes = [_c_p, ctypes.c_int, _c_p, _c_p, _c_p, ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_batch_bind.argtypes = [_c_p, _c_p, ctypes.c_size_t, _c_p]
    lib.ssa_batch_solve.argtypes = [_c_p, ctypes.c_int, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p,
                                    _c_p]
    lib.ssa_batch_profile_enable.argtypes = [_c_p, ctypes.c_uint]
    lib.ssa_batch_profile_read.argtypes = [_c_p, ctypes.c_int, ctypes.POINTER(_c_ll), ctypes.POINTER(ctypes.c_double)]
    lib.ssa_batch_destroy.argtypes = [_c_p]
    lib.ssa_batch_destroy.restype = None
    lib.ssa_server_create.argtypes = [_c_ll, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SsaOpts), _c_p,
                                      ctypes.c_size_t, _c_p, ctypes.POINTER(_c_p)]
    lib.ssa_server_enable_long.argtypes = [_c_p, _c_ll, ctypes.c_int]
    lib.ssa_server_create_stub.argtypes = [_c_ll, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SsaOpts), ctypes.c_size_t,
                                           ctypes.c_int, ctypes.POINTER(_c_p)]
    lib.ssa_server_request_bytes.argtypes = [_c_p, _c_ll, _c_ll, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_server_submit.argtypes = [_c_p, _c_ll, ctypes.c_ulonglong, _c_p, _c_ll, _c_ll, ctypes.c_int, _c_p, _c_p,
                                      _c_p, _c_p, _c_p]
    lib.ssa_server_step.argtypes = [_c_p, ctypes.POINTER(_c_ll), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.ssa_server_status.argtypes = [_c_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_hmatrix_workspace.argtypes = [_c_ll, _c_ll, _c_ll, _c_ll, _c_p, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_hmatrix.argtypes = [_c_p, _c_ll, _c_ll, _c_ll, _c_ll, _c_p, ctypes.c_int, _c_p, ctypes.c_size_t, _c_p,
                                _c_p]
    lib.ssa_realizations_workspace.argtypes = [_c_ll, _c_ll, _c_ll, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_realizations.argtypes = [_c_p, _c_ll, _c_ll, _c_ll, ctypes.c_int, _c_p, _c_p, ctypes.c_size_t, _c_p,
                                     _c_p, _c_p, _c_p]
    lib.ssa_server_destroy.argtypes = [_c_p]
    lib.ssa_server_destroy.restype = None
    lib.ssa_tune_workspace.argtypes = [_c_ll, _c_ll, ctypes.POINTER(ctypes.c_size_t)]
    lib.ssa_tune_fft.argtypes = [_c_ll, _c_ll, _c_p, _c_p, ctypes.c_size_t, _c_p, ctypes.c_int,
                                 ctypes.POINTER(SsaOpts), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                 ctypes.POINTER(_c_ll), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    for name in EXPORTED:
        if name not in ("ssa_plan_destroy", "ssa_status_str", "ssa_batch_destroy", "ssa_server_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(code: int) -> str:
    try:
        return load().ssa_status_str(int(code)).decode()
    except RuntimeError:
        return "library not loaded"


def _check(rc: int, where: str, allow_warn: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_warn):
        raise SsaError(rc, where)
    return rc


def bidiag_ritz(alpha, beta, d: int, k: int, vectors: bool = False):
    """Host utility: Ritz values (and optionally vectors) of the Lanczos bidiagonal B_d."""
    import numpy as np
    lib = load()
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    om = np.zeros(k)
    res = np.zeros(k)
    dp = ctypes.POINTER(ctypes.c_double)
    P = np.zeros((d + 1, k)) if vectors else None
    Q = np.zeros((d, k)) if vectors else None
    rc = lib.ssa_bidiag_ritz(a.ctypes.data_as(dp), b.ctypes.data_as(dp), d, k, om.ctypes.data_as(dp),
                             res.ctypes.data_as(dp), P.ctypes.data_as(dp) if vectors else None,
                             Q.ctypes.data_as(dp) if vectors else None)
    _check(rc, "ssa_bidiag_ritz")
    return (om, res, P, Q) if vectors else (om, res)


def dense_ritz(A, k: int):
    """Host utility: the k largest singular triples of a dense matrix (rows >= columns)."""
    import numpy as np
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    nr, nc = A.shape
    om = np.zeros(k)
    P = np.zeros((nr, k))
    Q = np.zeros((nc, k))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.ssa_dense_ritz(A.ctypes.data_as(dp), nr, nc, k, om.ctypes.data_as(dp), P.ctypes.data_as(dp),
                              Q.ctypes.data_as(dp)), "ssa_dense_ritz")
    return om, P, Q


class Plan:
    """One series geometry (N, L) bound to a torch-allocated device workspace."""

    def __init__(self, N: int, L: int, k_max: int, d_max: int = 0, check_every: int = 0,
                 tol: float = 0.0, seed: int = 0, device=None, stream=None, fft_m1: int = 0, fft_cb: int = 0,
                 restart_keep: int = 0, reorth: int = 0, fft_mp: int = 0, unfused: int = 0):
        import torch
        self._torch = torch
        lib = load()
        self.lib = lib
        self.N, self.L, self.K = int(N), int(L), int(N) - int(L) + 1
        self.k_max = int(k_max)
        opts = SsaOpts(int(d_max), int(check_every), float(tol), int(seed), int(fft_m1), int(fft_cb),
                       int(restart_keep), int(reorth), int(fft_mp), int(unfused))
        ws = ctypes.c_size_t(0)
        h = _c_p()
        _check(self._create(opts, ws, h), "ssa_embed_plan")
        self._h = h
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(int(ws.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib.ssa_plan_bind(h, base + off, int(ws.value), self.stream.cuda_stream), "ssa_plan_bind")
        d = SsaPlanDesc()
        _check(lib.ssa_plan_describe(h, ctypes.byref(d)), "ssa_plan_describe")
        self.desc = d

    def _create(self, opts, ws, h):
        return self.lib.ssa_embed_plan(self.N, self.L, self.k_max, ctypes.byref(opts), ctypes.byref(ws),
                                       ctypes.byref(h))

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ssa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, classes=None, on: bool = True, every: int = 1):
        """Count launches/bytes of every class and time the listed classes (all if None)
        with HIP events, one launch in `every`; on=False stops.  Clears the counters."""
        _check(self.lib.ssa_profile_sample(self._h, int(every)), "ssa_profile_sample")
        if not on:
            mask = 0
        elif classes is None:
            mask = (1 << len(PROF_CLASSES)) - 1
        else:
            mask = 0
            for c in classes:
                mask |= 1 << PROF_CLASSES.index(c)
        _check(self.lib.ssa_profile_enable(self._h, mask), "ssa_profile_enable")

    def profile_read(self):
        """{class: (launches, event-timed ms, algorithmic bytes)} since profile_enable."""
        out = {}
        for i, name in enumerate(PROF_CLASSES):
            n = _c_ll(0)
            ms = ctypes.c_double(0)
            b = ctypes.c_double(0)
            _check(self.lib.ssa_profile_read(self._h, i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
                   "ssa_profile_read")
            out[name] = (int(n.value), float(ms.value), float(b.value))
        return out

    def _series(self, f):
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if f.numel() != self.N:
            raise ValueError("series length differs from the plan")
        return f

    def embed(self, f):
        f = self._series(f)
        self._keep = f
        _check(self.lib.ssa_embed(self._h, f.data_ptr()), "ssa_embed")

    def matvec(self, x, transpose: bool = False):
        """X x (x has K entries) or X^T x (x has L entries), FP32 on the device."""
        torch = self._torch
        n_in = self.L if transpose else self.K
        n_out = self.K if transpose else self.L
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        if x.numel() != n_in:
            raise ValueError("vector length does not match")
        y = torch.empty(n_out, dtype=torch.float32, device=self.device)
        _check(self.lib.ssa_matvec(self._h, 1 if transpose else 0, x.data_ptr(), y.data_ptr()), "ssa_matvec")
        return y

    def truncated_svd(self, f, k: int):
        """Returns (sigma [k] f64, U [k, L] f32, V [k, K] f32, info); row i of U is u_i."""
        torch = self._torch
        f = self._series(f)
        sigma = torch.empty(k, dtype=torch.float64, device=self.device)
        U = torch.empty((k, self.L), dtype=torch.float32, device=self.device)
        V = torch.empty((k, self.K), dtype=torch.float32, device=self.device)
        info = SsaInfo()
        rc = self.lib.ssa_truncated_svd(self._h, f.data_ptr(), self.N, self.L, int(k), sigma.data_ptr(),
                                        U.data_ptr(), V.data_ptr(), ctypes.byref(info))
        _check(rc, "ssa_truncated_svd", allow_warn=True)
        return sigma, U, V, info

    def reconstruct(self, sigma, U, V, groups):
        """One series per group of triple indices; returns an (m, N) float32 tensor."""
        torch = self._torch
        k = int(sigma.numel())
        offs = [0]
        mem: list[int] = []
        for g in groups:
            mem.extend(int(i) for i in g)
            offs.append(len(mem))
        m = len(groups)
        offs_a = (ctypes.c_int * len(offs))(*offs)
        mem_a = (ctypes.c_int * max(1, len(mem)))(*(mem if mem else [0]))
        out = torch.empty((m, self.N), dtype=torch.float32, device=self.device)
        rc = self.lib.ssa_reconstruct(self._h, sigma.data_ptr(), U.contiguous().data_ptr(),
                                      V.contiguous().data_ptr(), k, ctypes.cast(offs_a, _c_p),
                                      ctypes.cast(mem_a, _c_p), m, out.data_ptr())
        _check(rc, "ssa_reconstruct")
        return out


def matvec_static(f, L: int, x, transpose: bool = False, device=None, stream=None):
    """X x (x has K entries) or X^T x (x has L entries) by ``ssa_matvec_static``: no plan and no
    workspace, the library's static device array holds every intermediate.  FP32 on the device."""
    import torch
    lib = load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    f = torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous()
    N, L = int(f.numel()), int(L)
    K = N - L + 1
    n_in, n_out = (L, K) if transpose else (K, L)
    x = torch.as_tensor(x, dtype=torch.float32, device=dev).contiguous()
    if x.numel() != n_in:
        raise ValueError("vector length does not match")
    y = torch.empty(max(n_out, 1), dtype=torch.float32, device=dev)
    _check(lib.ssa_matvec_static(_c_p(f.data_ptr()), N, L, 1 if transpose else 0, _c_p(x.data_ptr()),
                                 _c_p(y.data_ptr()), _c_p(st.cuda_stream)), "ssa_matvec_static")
    return y[:n_out]


def tune_fft(N: int, L: int, series=None, reps: int = 20, max_rows: int = 512, device=None, stream=None):
    """Time the FFT schedules of the products for (N, L) with ``ssa_tune_fft``.

    ``series`` (N values; zeros if None) is embedded for every candidate; the time per
    product pair does not depend on its values.  Returns (best, us_best, table): best is
    {"fft_mp", "fft_m1", "fft_cb"} to pass to Plan, us_best its microseconds per pair
    (X v and X^T u), and table a list of (M', M1, CB, us) for every candidate timed."""
    import torch
    lib = load()
    N, L = int(N), int(L)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    need = ctypes.c_size_t(0)
    _check(lib.ssa_tune_workspace(N, L, ctypes.byref(need)), "ssa_tune_workspace")
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    off = (-base) % 256
    if series is None:
        f = torch.zeros(N, dtype=torch.float64, device=dev)
    else:
        f = torch.as_tensor(series, dtype=torch.float64, device=dev).contiguous()
        if f.numel() != N:
            raise ValueError("series length differs from N")
    best = SsaOpts()
    us_best = ctypes.c_double(0)
    rows = (_c_ll * (3 * max(1, max_rows)))()
    us = (ctypes.c_double * max(1, max_rows))()
    nrows = ctypes.c_int(0)
    _check(lib.ssa_tune_fft(N, L, _c_p(f.data_ptr()), _c_p(base + off), int(need.value),
                            _c_p(st.cuda_stream), int(reps), ctypes.byref(best), ctypes.byref(us_best),
                            int(max_rows), rows, us, ctypes.byref(nrows)), "ssa_tune_fft")
    n = min(int(nrows.value), max_rows)
    table = [(int(rows[3 * i]), int(rows[3 * i + 1]), int(rows[3 * i + 2]), float(us[i])) for i in range(n)]
    return ({"fft_mp": int(best.fft_mp), "fft_m1": int(best.fft_m1), "fft_cb": int(best.fft_cb)},
            float(us_best.value), table)


class Plan2D(Plan):
    """2D-SSA of an Nx x Ny array with an Lx x Ly window (``ssa_embed_plan_2d``).  The array
    (row-major, any shape with Nx*Ny values) is the series; row i of U is the i-th Lx x Ly
    eigen-array, row i of V a Kx x Ky one, both flattened row by row; ``reconstruct`` returns
    (m, Nx, Ny)."""

    def __init__(self, Nx: int, Ny: int, Lx: int, Ly: int, k_max: int, **kw):
        self.Nx, self.Ny, self.Lx, self.Ly = int(Nx), int(Ny), int(Lx), int(Ly)
        self.Kx, self.Ky = self.Nx - self.Lx + 1, self.Ny - self.Ly + 1
        super().__init__(self.Nx * self.Ny, self.Lx * self.Ly, k_max, **kw)
        self.K = self.Kx * self.Ky

    def _create(self, opts, ws, h):
        return self.lib.ssa_embed_plan_2d(self.Nx, self.Ny, self.Lx, self.Ly, self.k_max, ctypes.byref(opts),
                                          ctypes.byref(ws), ctypes.byref(h))

    def reconstruct(self, sigma, U, V, groups):
        return super().reconstruct(sigma, U, V, groups).view(len(groups), self.Nx, self.Ny)


class Batch:
    """Many independent series solved together (``ssa_batch_*``): lockstep launches,
    one workgroup per series.  The device workspace grows to what each solve needs."""

    def __init__(self, n_max: int, k_max: int, max_series: int, d_max: int = 0, check_every: int = 0,
                 tol: float = 0.0, seed: int = 0, device=None, stream=None, reorth: int = 0):
        import torch
        self._torch = torch
        lib = load()
        self.lib = lib
        opts = SsaOpts(int(d_max), int(check_every), float(tol), int(seed), 0, 0, 0, int(reorth))
        ws = ctypes.c_size_t(0)
        h = _c_p()
        _check(lib.ssa_batch_plan(int(n_max), int(k_max), int(max_series), ctypes.byref(opts),
                                  ctypes.byref(ws), ctypes.byref(h)), "ssa_batch_plan")
        self._h = h
        self.bound_bytes = int(ws.value)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = None
        self.ws_bytes = 0

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ssa_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _tables(self, series, L, k, keys):
        import numpy as np
        torch = self._torch
        parts = [torch.as_tensor(x, dtype=torch.float64, device=self.device).reshape(-1) for x in series]
        ns = len(parts)
        lens = np.array([int(p.numel()) for p in parts], dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        L = np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(ns))
        k = np.ascontiguousarray(np.asarray(k, dtype=np.int32).reshape(ns))
        keys = None if keys is None else np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(ns))
        return parts, lens, offs, L, k, keys

    def profile_enable(self, classes=None, on: bool = True):
        """Time the listed kernel classes (all if None) with HIP events; on=False stops."""
        if not on:
            mask = 0
        elif classes is None:
            mask = (1 << len(BATCH_PROF_CLASSES)) - 1
        else:
            mask = 0
            for c in classes:
                mask |= 1 << BATCH_PROF_CLASSES.index(c)
        _check(self.lib.ssa_batch_profile_enable(self._h, mask), "ssa_batch_profile_enable")

    def profile_read(self):
        """{class: (launches, ms or -1)} since the last profile_enable."""
        out = {}
        for i, c in enumerate(BATCH_PROF_CLASSES):
            n = _c_ll(0)
            ms = ctypes.c_double(0.0)
            _check(self.lib.ssa_batch_profile_read(self._h, i, ctypes.byref(n), ctypes.byref(ms)),
                   "ssa_batch_profile_read")
            out[c] = (int(n.value), float(ms.value))
        return out

    def workspace_bytes(self, lens, L, k):
        import numpy as np
        lens = np.asarray(lens, dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        L = np.ascontiguousarray(np.asarray(L, dtype=np.int32))
        k = np.ascontiguousarray(np.asarray(k, dtype=np.int32))
        need = ctypes.c_size_t(0)
        _check(self.lib.ssa_batch_workspace(self._h, len(lens), offs.ctypes.data, L.ctypes.data, k.ctypes.data,
                                            ctypes.byref(need)), "ssa_batch_workspace")
        return int(need.value)

    def solve(self, series, L, k, recon: bool = True, keys=None):
        """series: list of 1-D arrays/tensors; L, k (and optional keys): per-series lists.
        Returns a dict of per-series views: sigma[s] (k_s,), U[s] (k_s, L_s), V[s] (k_s, K_s),
        recon[s] (k_s, N_s) and info (nseries, 4): steps, converged, restarts, DGKS passes."""
        torch = self._torch
        parts, lens, offs, L, k, keys = self._tables(series, L, k, keys)
        ns = len(parts)
        need = self.workspace_bytes(lens, L, k)
        if need > self.ws_bytes:
            self.workspace = None
            self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            _check(self.lib.ssa_batch_bind(self._h, base + (-base) % 256, need, self.stream.cuda_stream),
                   "ssa_batch_bind")
            self.ws_bytes = need
        flat = torch.cat(parts).contiguous()
        K = lens - L + 1
        sig = torch.empty(int(k.sum()), dtype=torch.float64, device=self.device)
        U = torch.empty(int((L * k).sum()), dtype=torch.float32, device=self.device)
        V = torch.empty(int((K * k).sum()), dtype=torch.float32, device=self.device)
        R = torch.empty(int((lens * k).sum()), dtype=torch.float32, device=self.device) if recon else None
        info = torch.zeros((ns, 4), dtype=torch.int32, device=self.device)
        rc = self.lib.ssa_batch_solve(self._h, ns, flat.data_ptr(), offs.ctypes.data, L.ctypes.data,
                                      k.ctypes.data, keys.ctypes.data if keys is not None else None,
                                      sig.data_ptr(), U.data_ptr(), V.data_ptr(),
                                      R.data_ptr() if recon else None, info.data_ptr())
        _check(rc, "ssa_batch_solve")
        self._keep = (flat, offs, L, k, keys)
        out = {"sigma": [], "U": [], "V": [], "recon": [] if recon else None, "info": info}
        so = uo = vo = ro = 0
        for s in range(ns):
            ks, Ls, Ks, Ns = int(k[s]), int(L[s]), int(K[s]), int(lens[s])
            out["sigma"].append(sig[so:so + ks])
            out["U"].append(U[uo:uo + Ls * ks].view(ks, Ls))
            out["V"].append(V[vo:vo + Ks * ks].view(ks, Ks))
            if recon:
                out["recon"].append(R[ro:ro + Ns * ks].view(ks, Ns))
            so += ks
            uo += Ls * ks
            vo += Ks * ks
            ro += Ns * ks
        return out


class Server:
    """Continuous batching of SSA requests (``ssa_server_*``): a device pool of
    ``pool_bytes`` (the HBM budget), ``slots`` batched requests (N <= n_max) in flight,
    one Lanczos step of every admitted one per tick; with ``long_slots`` > 0 also up to
    that many longer requests (N <= n_long_max), each advanced one check interval per tick
    on a plan bound to its pool region."""

    def __init__(self, n_max: int, k_max: int, slots: int, pool_bytes: int, d_max: int = 0,
                 check_every: int = 0, tol: float = 0.0, seed: int = 0, device=None, stream=None, reorth: int = 0,
                 n_long_max: int = 0, long_slots: int = 0):
        import torch
        self._torch = torch
        lib = load()
        self.lib = lib
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.pool.data_ptr()
        opts = SsaOpts(int(d_max), int(check_every), float(tol), int(seed), 0, 0, 0, int(reorth))
        h = _c_p()
        _check(lib.ssa_server_create(int(n_max), int(k_max), int(slots), ctypes.byref(opts), base + (-base) % 256,
                                     int(pool_bytes), self.stream.cuda_stream, ctypes.byref(h)), "ssa_server_create")
        self._h = h
        self.slots = int(slots) + int(long_slots)
        self.n_max = int(n_max)
        self._live = {}
        if long_slots:
            _check(lib.ssa_server_enable_long(h, int(n_long_max), int(long_slots)), "ssa_server_enable_long")

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ssa_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def request_bytes(self, N: int, L: int, k: int) -> int:
        b = ctypes.c_size_t(0)
        _check(self.lib.ssa_server_request_bytes(self._h, int(N), int(L), int(k), ctypes.byref(b)),
               "ssa_server_request_bytes")
        return int(b.value)

    def submit(self, rid: int, f, L: int, k: int, key: int | None = None, recon: bool = True):
        """Queue request ``rid``; returns its output tensors (valid once it completes)."""
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        N = int(f.numel())
        K = N - int(L) + 1
        out = {
            "f": f,
            "sigma": torch.empty(k, dtype=torch.float64, device=self.device),
            "U": torch.empty((k, int(L)), dtype=torch.float32, device=self.device),
            "V": torch.empty((k, K), dtype=torch.float32, device=self.device),
            "recon": torch.empty((k, N), dtype=torch.float32, device=self.device) if recon else None,
            "info": torch.zeros(4, dtype=torch.int32, device=self.device),
        }
        if N > self.n_max:  # solved on a stream of its own: the inputs and outputs must be ready
            torch.cuda.current_stream(self.device).synchronize()
        _check(self.lib.ssa_server_submit(self._h, int(rid), int(rid if key is None else key), f.data_ptr(), N,
                                          int(L), int(k), out["sigma"].data_ptr(), out["U"].data_ptr(),
                                          out["V"].data_ptr(), out["recon"].data_ptr() if recon else None,
                                          out["info"].data_ptr()), "ssa_server_submit")
        self._live[int(rid)] = out
        return out

    def step(self):
        """One tick; returns the list of (id, outputs) completed."""
        buf = (_c_ll * self.slots)()
        n = ctypes.c_int(0)
        _check(self.lib.ssa_server_step(self._h, buf, self.slots, ctypes.byref(n)), "ssa_server_step")
        return [(int(buf[i]), self._live.pop(int(buf[i]))) for i in range(n.value)]

    def status(self):
        q, a, f = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        free = ctypes.c_size_t(0)
        _check(self.lib.ssa_server_status(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(f),
                                          ctypes.byref(free)), "ssa_server_status")
        return {"queued": q.value, "active": a.value, "finalizing": f.value, "pool_free": int(free.value)}


def hmatrix(f, B: int, T: int, L: int, I, device=None, stream=None):
    """H-matrix of heterogeneity indices (structural-change detection) of a series on the
    GPU: base windows of length B, test windows of length T, window L, 1-based index set I.
    Returns an (N-B+1, N-T+1) FP64 tensor."""
    import numpy as np
    import torch
    lib = load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    f = torch.as_tensor(f, dtype=torch.float64, device=dev).reshape(-1).contiguous()
    N = int(f.numel())
    Ia = np.ascontiguousarray(np.asarray(I, dtype=np.int32))
    need = ctypes.c_size_t(0)
    _check(lib.ssa_hmatrix_workspace(N, int(B), int(T), int(L), Ia.ctypes.data, Ia.size, ctypes.byref(need)),
           "ssa_hmatrix_workspace")
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    G = torch.empty((N - int(B) + 1, N - int(T) + 1), dtype=torch.float64, device=dev)
    _check(lib.ssa_hmatrix(f.data_ptr(), N, int(B), int(T), int(L), Ia.ctypes.data, Ia.size, base + (-base) % 256,
                           int(need.value), st.cuda_stream, G.data_ptr()), "ssa_hmatrix")
    return G


def realizations(F, L: int, d: int, truth=None, device=None, stream=None):
    """Repeated realizations on the GPU: rows of F (R x N) reconstructed from their first d
    eigentriples; returns (mean, var, mse or None) per point as FP64 tensors."""
    import torch
    lib = load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    F = torch.as_tensor(F, dtype=torch.float64, device=dev).contiguous()
    R, N = F.shape
    need = ctypes.c_size_t(0)
    _check(lib.ssa_realizations_workspace(R, N, int(L), int(d), ctypes.byref(need)), "ssa_realizations_workspace")
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    mean = torch.empty(N, dtype=torch.float64, device=dev)
    var = torch.empty(N, dtype=torch.float64, device=dev)
    tr = torch.as_tensor(truth, dtype=torch.float64, device=dev).contiguous() if truth is not None else None
    mse = torch.empty(N, dtype=torch.float64, device=dev) if truth is not None else None
    _check(lib.ssa_realizations(F.data_ptr(), R, N, int(L), int(d), tr.data_ptr() if tr is not None else None,
                                base + (-base) % 256, int(need.value), st.cuda_stream, mean.data_ptr(),
                                var.data_ptr(), mse.data_ptr() if mse is not None else None), "ssa_realizations")
    return mean, var, mse
