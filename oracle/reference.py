"""Reference solution x*_ref, the direct baseline and the effective dimension.

Test infrastructure only.

* ``direct_solve``: the paper's direct baseline (Sec. 5): form H = A^T A + nu^2 Lambda and
  solve by Cholesky, in FP64.
* ``reference_solution``: x* = H^{-1} b, the plain definition of the result, to near FP64
  accuracy: a first solve, then iterative refinement x <- x + C^{-1} r whose residual
  r = b - A^T (A x) - nu^2 Lambda x is evaluated in extended precision (x86 long double,
  64-bit significand).  The fixed point depends only on (A, b, nu, Lambda); the correction
  operator C^{-1} only sets the speed: the Cholesky factor of the FP64-formed H, or, for
  synthetic A = U diag(sigma) V^T with Lambda = I, the spectral inverse
  V diag(1/(sigma^2 + nu^2)) V^T.
* ``effective_dimension``: d_e = tr(A_nu) / ||A_nu||_2 with A_nu = A^T A (A^T A + nu^2
  Lambda)^{-1} (Sec. 1, Notations), computed from eigenvalues.
  ``effective_dimension_closed``: the same for A = U diag(sigma) V^T and Lambda = I:
  sum_j s_j / max_j s_j with s_j = sigma_j^2 / (sigma_j^2 + nu^2); ``effective_dimension_sum``
  is the plain sum_j s_j.

Pins (tests/test_oracle_reference.py): x*_ref == numpy.linalg.solve on tiny inputs; the
refined solution has an extended-precision residual at rounding level; both correction
operators converge to the same x; d_e by eigenvalues == closed form.
"""
import concurrent.futures as cf
import os

import numpy as np
import scipy.linalg as sla


def _rows_chunks(n, chunk):
    return [(i, min(n, i + chunk)) for i in range(0, n, chunk)]


def residual_extended(A, b, nu, lam, x, chunk=2048, threads=None):
    """b - A^T (A x) - nu^2 Lambda x accumulated in long double; returned as long double.

    Each block of rows contributes A_blk^T (A_blk x) in long double; block contributions are
    summed in a fixed order.
    """
    A = np.asarray(A)
    n, d = A.shape
    X = np.asarray(x, dtype=np.float64)
    squeeze = X.ndim == 1
    X2 = X[:, None] if squeeze else X
    xl = X2.astype(np.longdouble)
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)

    def part(rng):
        i0, i1 = rng
        Al = A[i0:i1].astype(np.longdouble)
        z = Al @ xl
        return Al.T @ z

    chunks = _rows_chunks(n, chunk)
    threads = threads or min(16, os.cpu_count() or 1)
    acc = np.zeros(X2.shape, dtype=np.longdouble)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for contrib in ex.map(part, chunks):
            acc += contrib
    B = np.asarray(b, dtype=np.float64)
    B2 = (B[:, None] if B.ndim == 1 else B).astype(np.longdouble)
    nu2 = np.longdouble(nu) * np.longdouble(nu)
    r = B2 - acc - nu2 * lam.astype(np.longdouble)[:, None] * xl
    return r[:, 0] if squeeze else r


def direct_solve(A, b, nu, lam=None):
    """Paper's direct baseline: Cholesky of the formed H (FP64)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    H = A.T @ A + (nu ** 2) * np.diag(lam)
    cf_ = sla.cho_factor(H, lower=True)
    return sla.cho_solve(cf_, np.asarray(b, dtype=np.float64))


def reference_solution(A, b, nu, lam=None, spectral=None, max_refine=10, rtol=1e-17, return_history=False):
    """x*_ref = H^{-1} b by refined direct solve (see module docstring).

    spectral: optional (V, sigma) of A = U diag(sigma) V^T, used as the correction operator
    when Lambda = I (avoids forming A^T A at large n).
    """
    A = np.asarray(A)
    d = A.shape[1]
    lam_v = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    if spectral is not None and np.all(lam_v == 1.0):
        V, sigma = spectral
        V = np.asarray(V, dtype=np.float64)
        w = 1.0 / (np.asarray(sigma, dtype=np.float64) ** 2 + nu ** 2)

        def corr(r):
            return V @ ((w if r.ndim == 1 else w[:, None]) * (V.T @ r))
    else:
        H = A.T @ A + (nu ** 2) * np.diag(lam_v)
        cf_ = sla.cho_factor(H, lower=True)

        def corr(r):
            return sla.cho_solve(cf_, r)

    B = np.asarray(b, dtype=np.float64)
    x = corr(B)
    hist = []
    for _ in range(max_refine):
        r = residual_extended(A, B, nu, lam_v, x).astype(np.float64)
        dx = corr(r)
        x = x + dx
        num = np.linalg.norm(dx, axis=0)
        den = np.linalg.norm(x, axis=0)
        rel = float(np.max(num / np.where(den > 0, den, 1.0)))
        hist.append(rel)
        if rel <= rtol or (len(hist) >= 2 and hist[-1] >= hist[-2] and rel < 1e-15):
            break
    return (x, hist) if return_history else x


def rel_error(x, xref):
    """Per-column ||x - x_ref||_2 / ||x_ref||_2 (a scalar for vectors)."""
    x = np.asarray(x, dtype=np.float64)
    xref = np.asarray(xref, dtype=np.float64)
    num = np.linalg.norm(x - xref, axis=0)
    den = np.linalg.norm(xref, axis=0)
    return num / den


def h_norm_error(A, nu, lam, x, xref):
    """delta_x = 1/2 ||x - x*||_H^2 (Sec. 1.1)."""
    e = np.asarray(x, dtype=np.float64) - np.asarray(xref, dtype=np.float64)
    lam = np.ones(A.shape[1]) if lam is None else np.asarray(lam, dtype=np.float64)
    Ae = A @ e
    return 0.5 * (np.sum(Ae * Ae, axis=0) + nu ** 2 * np.sum(lam.reshape(-1, *([1] * (e.ndim - 1))) * e * e, axis=0))


def effective_dimension(A, nu, lam=None):
    """d_e = tr(A_nu) / ||A_nu||_2, A_nu = A^T A (A^T A + nu^2 Lambda)^{-1} (Notations)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    G = A.T @ A
    # A_nu is similar to the symmetric M = H^{-1/2} G H^{-1/2}; its eigenvalues are those of
    # the generalized problem G v = mu H v.
    mu = sla.eigh(G, G + (nu ** 2) * np.diag(lam), eigvals_only=True)
    return float(np.sum(mu) / np.max(mu))


def effective_dimension_closed(sigma, nu):
    s = np.asarray(sigma, dtype=np.float64) ** 2
    r = s / (s + nu ** 2)
    return float(np.sum(r) / np.max(r))


def effective_dimension_sum(sigma, nu):
    s = np.asarray(sigma, dtype=np.float64) ** 2
    return float(np.sum(s / (s + nu ** 2)))
