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
