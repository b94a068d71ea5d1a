"""Comparison rules between the HIP path and the FP64 oracle.

Tolerances (FP32 products, FP64 Lanczos scalars):
  * singular values: relative error <= 1e-5 for sigma_i >= 1e-2 sigma_1; below
    that, absolute error <= 1e-7 sigma_1 (the size of the FP32 rounding of one
    product X v, which bounds what any FP32 matvec can resolve);
  * vectors: largest principal-angle sine <= 1e-4 per cluster, because
    individual vectors inside a cluster are not unique.  Two neighbouring
    values belong to one cluster when their gap is below
        max(1e-3 sigma_i, DELTA / 1e-4),   DELTA = 16 u |X|_F,  u = 2^-24,
    i.e. when Wedin's bound sin(theta) <= |E| / gap cannot certify 1e-4 for a
    perturbation E of the size the FP32 path itself introduces (rounding the
    series to FP32 alone is a Hankel perturbation with |E| <= u |X|_F; the FFT
    products and FP32 vector storage add errors of the same order);
  * reconstructions: max-abs error <= 1e-5 |F|_inf per isolated triple, and per
    cluster (sum over the cluster) otherwise.
A cluster that straddles k (its last member beyond k) is compared by its
singular values only.
"""
import numpy as np

SIGMA_REL = 1e-5
SIGMA_FLOOR = 1e-7
ANGLE_SIN = 1e-4
RECON_REL = 1e-5
CLUSTER_GAP = 1e-3
U32 = 2.0 ** -24
BACKWARD = 16.0 * U32


def frobenius(f, L):
    """|X|_F of the trajectory matrix: each f[n] appears on cnt[n] antidiagonal entries."""
    f = np.asarray(f, dtype=np.float64)
    N = f.size
    K = N - L + 1
    n = np.arange(N)
    cnt = np.minimum.reduce([n + 1, np.full(N, L), np.full(N, K), N - n])
    return float(np.sqrt(np.sum(cnt * f * f)))


def clusters(s_ref, k, fro=None):
    """Index groups of near-equal oracle singular values among the first k
    (s_ref may hold more than k values so straddling clusters are visible).
    fro = |X|_F enables the FP32-conditioning part of the rule."""
    wedin_gap = 0.0 if fro is None else BACKWARD * fro / ANGLE_SIN
    out, i = [], 0
    while i < k:
        j = i + 1
        while (j < len(s_ref) and s_ref[j - 1] > 0
               and (s_ref[j - 1] - s_ref[j]) < max(CLUSTER_GAP * s_ref[j - 1], wedin_gap)):
            j += 1
        out.append(list(range(i, min(j, len(s_ref)))))
        i = j
    return out


def sigma_errors(s_gpu, s_ref):
    s_gpu = np.asarray(s_gpu, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)[: len(s_gpu)]
    s1 = s_ref[0]
    err = np.abs(s_gpu - s_ref)
    bound = np.where(s_ref >= 1e-2 * s1, SIGMA_REL * s_ref, SIGMA_FLOOR * s1)
    return err, bound


def assert_sigma(s_gpu, s_ref):
    err, bound = sigma_errors(s_gpu, s_ref)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, f"sigma mismatch at {bad}: gpu={np.asarray(s_gpu)[bad]} ref={np.asarray(s_ref)[bad]}"
    return float(np.max(err / np.maximum(np.asarray(s_ref)[: len(err)], 1e-300)))


def subspace_sin(A, B):
    qa, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    qb, _ = np.linalg.qr(np.asarray(B, dtype=np.float64))
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))


def compare_svd(s_gpu, U_gpu, V_gpu, s_ref, U_ref, V_ref, k, fro=None, min_rel=1e-6):
    """U/V as (n, k) arrays (columns = vectors).  Returns a report dict; asserts."""
    worst_sin = 0.0
    rel = assert_sigma(s_gpu[:k], s_ref[:k])
    for c in clusters(s_ref, k, fro):
        if max(c) >= k:
            continue  # straddles k: sigma only
        if s_ref[c[0]] <= min_rel * s_ref[0]:
            continue  # null space: vectors arbitrary
        su = subspace_sin(U_ref[:, c], U_gpu[:, c])
        sv = subspace_sin(V_ref[:, c], V_gpu[:, c])
        worst_sin = max(worst_sin, su, sv)
        assert su <= ANGLE_SIN and sv <= ANGLE_SIN, f"cluster {c}: sin(theta) u={su:.2e} v={sv:.2e}"
    return {"sigma_rel": rel, "sin_theta": worst_sin}


def compare_recon(rec_gpu, rec_ref, f_inf):
    err = float(np.max(np.abs(np.asarray(rec_gpu, dtype=np.float64) - rec_ref)))
    assert err <= RECON_REL * f_inf, f"reconstruction error {err:.3e} > {RECON_REL * f_inf:.3e}"
    return err
