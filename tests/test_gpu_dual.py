"""Dual form (n < d, Sec. 1): parity of aes_solve_dual against the oracle's dual route."""
import math

import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
from oracle import reference, solvers

from _helpers import to_dev

pytestmark = pytest.mark.gpu


def _problem(n, d, c, seed, with_lam=True, decay=0.9):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, d)) / math.sqrt(d) * (decay ** np.arange(n))[:, None]
    lam = 1.0 + rng.random(d) if with_lam else None
    b = rng.standard_normal((d, c)) if c > 1 else rng.standard_normal(d)
    return A, b, lam


def _dual(A, b, lam, nu, **kw):
    return aes.solve_dual(to_dev(A), to_dev(b), nu, to_dev(lam) if lam is not None else None, **kw)


def _traj(info):
    return [(e["t"], e["m"], e["accept"]) for e in info["trace"]]


@pytest.mark.parametrize("method,sketch", [("pcg", "srht"), ("ihs", "srht"), ("pcg", "sjlt")])
def test_dual_trajectory_and_accuracy(method, sketch):
    # n = 40 unknowns in the dual, d = 1500 rows of B = Lambda^{-1/2} A^T (a ragged 2048 pad)
    A, b, lam = _problem(40, 1500, 1, 1)
    nu = 0.05
    kw = dict(method=method, sketch=sketch, m_init=8, seed=3, tol=1e-11)
    x, info = _dual(A, b, lam, nu, trace_cap=256, **kw)
    xo, wo, io = solvers.dual_solve(A, b, nu, lam, solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj(info) == [(e["t"], e["m"], bool(e["accept"])) for e in io.trace]
    assert info["iterations"] == io.iterations and info["final_m"] == io.final_m
    assert info["a_passes"] == io.a_passes
    xr = reference.reference_solution(A, b, nu, lam)
    assert reference.rel_error(x.cpu().numpy(), xr) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9


def test_dual_fixed_steps_match_the_oracle_iterate():
    # three accepted steps, not converged: the map back x = Lambda^{-1} (b - A^T w) / nu^2 is
    # checked on an iterate that is far from x*
    A, b, lam = _problem(64, 3000, 1, 2)
    nu = 0.02
    kw = dict(method="pcg", sketch="srht", m_init=16, seed=5, stop="fixed", max_iter=3, adaptive=False, tol=1e-10)
    x, info = _dual(A, b, lam, nu, **kw)
    xo, wo, io = solvers.dual_solve(A, b, nu, lam, solvers.Options(**kw))
    assert info["iterations"] == io.iterations == 3
    xr = reference.reference_solution(A, b, nu, lam)
    assert reference.rel_error(xo, xr) > 1e-6  # really an intermediate iterate
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-10


@pytest.mark.parametrize("sketch,with_lam", [("srht", False), ("gauss", True), ("sjlt", True)])
def test_dual_several_rhs(sketch, with_lam):
    A, b, lam = _problem(48, 2000, 3, 3, with_lam=with_lam)
    nu = 0.1
    X, info = _dual(A, b, lam, nu, sketch=sketch, m_init=8, seed=1, tol=1e-11)
    assert info["status"] == "ok" and X.shape == (2000, 3)
    Xr = reference.reference_solution(A, b, nu, lam)
    assert np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)
    # a strided output: only the c columns of x are written
    out = torch.full((2000, 5), 7.0, dtype=torch.float64, device=X.device)
    _dual(A, b, lam, nu, sketch=sketch, m_init=8, seed=1, tol=1e-11, x=out[:, :3])
    assert torch.equal(out[:, :3], X) and bool((out[:, 3:] == 7.0).all())


@pytest.mark.parametrize("precision", ["mixed", "mixed_fp32"])
def test_dual_mixed_precision(precision):
    # the dual solve in mixed precision (FP32 inner solves over B, FP64 refinement of w)
    A, b, lam = _problem(48, 2000, 3, 3)
    nu = 0.1
    X, info = _dual(A, b, lam, nu, precision=precision, m_init=8, seed=1, tol=1e-11)
    assert info["status"] == "ok", info
    Xr = reference.reference_solution(A, b, nu, lam)
    assert np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)


def test_dual_wider_than_the_primal_limit():
    # d = 40000 > 32768 (the primal entry point's limit); the dual has n = 256 unknowns
    A, b, lam = _problem(256, 40000, 1, 7, decay=0.95)
    nu = 0.05
    kw = dict(m_init=8, seed=2, tol=1e-10)
    dA, db, dlam = to_dev(A), to_dev(b), to_dev(lam)
    with pytest.raises(aes.AesError):
        aes.solve(dA, db, nu, dlam, **kw)
    x, info = aes.solve_dual(dA, db, nu, dlam, trace_cap=256, **kw)
    xo, wo, io = solvers.dual_solve(A, b, nu, lam, solvers.Options(**kw))
    assert info["status"] == "ok"
    assert info["final_m"] == io.final_m and info["iterations"] == io.iterations
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9
    # primal optimality at the returned x, in extended precision: ||b - H x|| small
    r = reference.residual_extended(A, b, nu, lam, x.cpu().numpy())
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)


def test_dual_validation_leaves_x_untouched():
    dev = torch.device("cuda:0")
    A = torch.zeros((32769, 1), dtype=torch.float64, device=dev)  # n above 32768
    b = torch.ones(1, dtype=torch.float64, device=dev)
    x = torch.full((1,), 3.0, dtype=torch.float64, device=dev)
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve_dual(A, b, 1.0, x=x)
    assert float(x[0]) == 3.0
    A2, b2, _ = _problem(8, 100, 1, 9)
    with pytest.raises(ValueError):
        aes.solve_dual(to_dev(A2), to_dev(b2), 1.0, x0=torch.zeros(8, dtype=torch.float64, device=dev))
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve_dual(to_dev(A2), to_dev(b2), -1.0)
