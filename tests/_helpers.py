"""Shared helpers of the GPU tests (inputs to device, tolerances)."""
import numpy as np
import torch

U = np.finfo(np.float64).eps / 2  # unit roundoff of FP64


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def hv_bound(A, lam, nu, p):
    """Componentwise rounding bound of q = A^T (A p) + nu^2 Lambda p in FP64 (Higham, gamma_k)."""
    n, d = A.shape
    absA = np.abs(A)
    lam = np.ones(d) if lam is None else lam
    mag = absA.T @ (absA @ np.abs(p)) + nu ** 2 * lam * np.abs(p)
    k = n + d + 8
    return 2 * k * U * mag / (1 - k * U)


def spectral_error(A, b, nu, V, sigma, x, threads=None):
    """Per-column ||x - x*|| / ||x|| for A = U diag(sigma) V^T (Lambda = I), from the oracle's
    extended-precision residual r = b - H x: x* - x = H^{-1} r, applied by the spectral inverse
    V diag(1 / (sigma^2 + nu^2)) V^T (exact for the ideal A; its relative error as an estimate
    of H^{-1} r is about kappa * 1e-16, far below the 1e-10 tested)."""
    from oracle import reference

    r = reference.residual_extended(A, b, nu, None, x, threads=threads).astype(np.float64)
    w = 1.0 / (np.asarray(sigma, dtype=np.float64) ** 2 + nu ** 2)
    e = V @ (w[:, None] * (V.T @ (r if r.ndim == 2 else r[:, None])))
    xx = x if x.ndim == 2 else x[:, None]
    return np.linalg.norm(e, axis=0) / np.linalg.norm(xx, axis=0)
