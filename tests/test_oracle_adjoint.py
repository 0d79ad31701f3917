"""Pins of the dense adjoint gradients: central finite differences (h = 1e-6, FP64)."""
import numpy as np

from oracle import adjoint


def _loss(A, b, nu, lam, xt):
    x, _ = adjoint.dense_solution(A, b, nu, lam)
    return adjoint.loss_half_sq(x, xt)[0]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    n, d, nu = 40, 6, 0.3
    A = rng.standard_normal((n, d)) * (0.7 ** np.arange(d))
    b = A.T @ rng.standard_normal(n)
    lam = 1 + rng.random(d)
    xt = rng.standard_normal(d)
    x, _ = adjoint.dense_solution(A, b, nu, lam)
    _, g = adjoint.loss_half_sq(x, xt)
    xs, adj, db, dA, dlognu = adjoint.gradients(A, b, nu, g, lam)
    h = 1e-6
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        fd = (_loss(A, b + e, nu, lam, xt) - _loss(A, b - e, nu, lam, xt)) / (2 * h)
        assert abs(fd - db[i]) <= 1e-6 * max(1.0, abs(db[i]))
    fd = (_loss(A, b, nu * np.exp(h), lam, xt) - _loss(A, b, nu * np.exp(-h), lam, xt)) / (2 * h)
    assert abs(fd - dlognu) <= 1e-6 * max(1.0, abs(dlognu))
    for _ in range(3):
        E = rng.standard_normal((n, d))
        fd = (_loss(A + h * E, b, nu, lam, xt) - _loss(A - h * E, b, nu, lam, xt)) / (2 * h)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
