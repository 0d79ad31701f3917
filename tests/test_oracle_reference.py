"""Pins of the reference solution, the direct baseline and the effective dimension."""
import numpy as np

import synth
from oracle import reference


def test_reference_equals_dense_solve_tiny():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((30, 5))
    lam = 1 + rng.random(5)
    b = rng.standard_normal(5)
    H = A.T @ A + 0.3 ** 2 * np.diag(lam)
    np.testing.assert_allclose(reference.reference_solution(A, b, 0.3, lam), np.linalg.solve(H, b), rtol=1e-14)
    np.testing.assert_allclose(reference.direct_solve(A, b, 0.3, lam), np.linalg.solve(H, b), rtol=1e-13)


def test_refinement_beats_direct_on_ill_conditioned():
    P = synth.make_problem(2048, 128, "geo:0.9", 1e-4, seed=3)
    A, b, nu = P["A"], P["b"], P["nu"]
    xr, hist = reference.reference_solution(A, b, nu, return_history=True)
    xs = reference.reference_solution(A, b, nu, spectral=(P["V"], P["sigma"]))
    assert np.max(reference.rel_error(xs, xr)) < 1e-13
    r_ref = np.abs(reference.residual_extended(A, b, nu, None, xr)).max()
    r_dir = np.abs(reference.residual_extended(A, b, nu, None, reference.direct_solve(A, b, nu))).max()
    assert r_ref < r_dir
    assert hist[-1] < 1e-13  # kappa(H) ~ 8e7: long-double residual limits the last digits


def test_effective_dimension_closed_form():
    for nu in (1e-1, 1e-2, 1e-3):
        P = synth.make_problem(1024, 96, "geo:0.95", nu, seed=1)
        de = reference.effective_dimension(P["A"], nu)
        assert abs(de - reference.effective_dimension_closed(P["sigma"], nu)) < 1e-8 * de
        assert reference.effective_dimension_sum(P["sigma"], nu) <= de <= 96


def test_residual_extended_matches_float_residual():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((500, 20))
    x = rng.standard_normal((20, 2))
    b = rng.standard_normal((20, 2))
    lam = 1 + rng.random(20)
    r = reference.residual_extended(A, b, 0.1, lam, x, chunk=64).astype(np.float64)
    np.testing.assert_allclose(r, b - A.T @ (A @ x) - 0.01 * lam[:, None] * x, rtol=1e-10, atol=1e-10)


def test_wide_problem_recipe():
    # n < d inputs of the dual form: A has exactly the prescribed n singular values, b = A^T y
    P = synth.make_wide_problem(200, 900, "geo:0.99", 1e-2, lam="uniform1_10", nrhs=2, seed=4)
    A = P["A"]
    assert A.shape == (200, 900) and P["b"].shape == (900, 2) and P["lam"].shape == (900,)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - P["sigma"]) / P["sigma"]) <= 1e-12
    assert np.allclose(P["b"], A.T @ P["y"], rtol=0, atol=1e-12)
    assert np.all((P["lam"] >= 1.0) & (P["lam"] <= 10.0))


def test_spectral_error_bound_matches_the_refined_reference():
    # the residual-based error of the GPU tests (extended residual, spectral inverse) equals the
    # error against the refined reference, for x far from and close to x*
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from _helpers import spectral_error

    P = synth.make_problem(3000, 96, "geo:0.98", 1e-4, nrhs=3, seed=8)
    xr = reference.reference_solution(P["A"], P["b"], P["nu"], spectral=(P["V"], P["sigma"]))
    rng = np.random.default_rng(1)
    for scale in (1e-3, 1e-9, 1e-12):
        x = xr * (1.0 + scale * rng.standard_normal(xr.shape))
        e_true = reference.rel_error(x, xr)
        e_est = spectral_error(P["A"], P["b"], P["nu"], P["V"], P["sigma"], x)
        np.testing.assert_allclose(e_est, e_true, rtol=1e-3)
