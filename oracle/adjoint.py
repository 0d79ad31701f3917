"""Dense FP64 gradients of a loss of the solution x* = H^{-1} b.  Test infrastructure only.

With H = A^T A + nu^2 Lambda symmetric, dx* = H^{-1} (db - dH x*) and
dH = dA^T A + A^T dA + 2 nu dnu Lambda.  For g = dL/dx* and the adjoint lam = H^{-1} g:

    dL/db     = lam
    dL/dA     = -(A x*) lam^T - (A lam) x*^T
    dL/dlognu = -2 nu^2 lam^T Lambda x*

Pins (tests/test_oracle_adjoint.py): central finite differences of the dense solve, entry by
entry for b and log(nu) and along random directions for A.
"""
import numpy as np
import scipy.linalg as sla


def dense_solution(A, b, nu, lam=None):
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    H = A.T @ A + (nu ** 2) * np.diag(lam)
    cf_ = sla.cho_factor(H, lower=True)
    return sla.cho_solve(cf_, np.asarray(b, dtype=np.float64)), cf_


def gradients(A, b, nu, g, lam=None, x=None):
    """(x*, adjoint, dL/db, dL/dA, dL/dlognu) for upstream gradient g = dL/dx*.

    If x is given it is used as x* (e.g. the refined reference) and only the adjoint solve
    is done here.
    """
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    xs, cf_ = dense_solution(A, b, nu, lam)
    if x is not None:
        xs = np.asarray(x, dtype=np.float64)
    adj = sla.cho_solve(cf_, np.asarray(g, dtype=np.float64))
    db = adj
    dA = -np.outer(A @ xs, adj) - np.outer(A @ adj, xs)
    dlognu = -2.0 * nu ** 2 * float(adj @ (lam * xs))
    return xs, adj, db, dA, dlognu


def loss_half_sq(x, xt):
    """L = 1/2 ||x - x_t||^2 and dL/dx."""
    e = np.asarray(x) - np.asarray(xt)
    return 0.5 * float(e @ e), e
