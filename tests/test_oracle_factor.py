"""Pins of the oracle's factorisation of H_S (Sec. 4.1): Cholesky and the Woodbury form."""
import numpy as np
import pytest

from oracle.factor import NotSPDError, SketchedHessian


@pytest.mark.parametrize("m,d", [(20, 8), (8, 8), (5, 12), (1, 9)])
def test_apply_equals_solve(m, d):
    rng = np.random.default_rng(m * 100 + d)
    SA = rng.standard_normal((m, d))
    lam = 1 + 9 * rng.random(d)
    nu = 0.3
    P = SketchedHessian(SA, nu, lam)
    assert P.woodbury == (m < d)
    HS = SA.T @ SA + nu ** 2 * np.diag(lam)
    z = rng.standard_normal((d, 3))
    np.testing.assert_allclose(P.apply(z), np.linalg.solve(HS, z), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(P.apply(z[:, 0]), np.linalg.solve(HS, z[:, 0]), rtol=1e-10, atol=1e-12)
    if not P.woodbury:
        np.testing.assert_allclose(P.L @ P.L.T, HS, rtol=1e-12, atol=1e-12)
    else:
        W = (SA / lam) @ SA.T + nu ** 2 * np.eye(m)
        np.testing.assert_allclose(P.L @ P.L.T, W, rtol=1e-12, atol=1e-12)


def test_not_spd_detected():
    SA = np.zeros((4, 3))
    with pytest.raises(NotSPDError):
        SketchedHessian(SA, 1.0, np.array([1.0, -2.0, 1.0]))
