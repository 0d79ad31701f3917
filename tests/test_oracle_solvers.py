"""Pins of the oracle's adaptive PCG (Algorithm 2) and adaptive IHS (Algorithm 1)."""
import math

import numpy as np
import pytest

import synth
from oracle import reference, solvers
from oracle import sketch as sk
from oracle.factor import SketchedHessian


def _tiny(n=64, d=8, nu=0.1, seed=0, lam=None):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, d)) * (0.6 ** np.arange(d))[None, :]
    b = A.T @ rng.standard_normal(n)
    lam = np.ones(d) if lam is None else lam
    return A, b, nu, lam


def _H(A, nu, lam):
    return A.T @ A + nu ** 2 * np.diag(lam)


def test_constants_limits():
    # PCG rate phi(rho) ~ rho/4 for small rho and is below the IHS rate rho (Sec. 3.2).
    for rho in (1e-4, 0.01, 0.125, 0.5):
        phi, c = solvers.pcg_constants(rho)
        assert 0 < phi < rho
        assert c > 4
    phi, c = solvers.pcg_constants(1e-6)
    assert abs(phi / 1e-6 - 0.25) < 1e-3
    assert abs(c - 4) < 0.02  # c(alpha, rho) -> alpha = 4, the constant of the PCG rate bound
    phi_i, c_i, mu = solvers.ihs_constants(1e-6)
    assert phi_i == 1e-6 and abs(c_i - 1) < 0.005 and mu == 1 - 1e-6


def test_pcg_one_step_when_sketch_is_full():
    A, b, nu, lam = _tiny(n=60, d=7)
    o = solvers.Options(m_init=64, adaptive=False, stop="fixed", max_iter=1, seed=3)
    x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    xs = np.linalg.solve(_H(A, nu, lam), b)
    assert info.iterations == 1
    assert reference.rel_error(x, xs) < 1e-12


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5])
def test_pcg_krylov_optimality(t):
    # Theorem "rate cg": PCG's x_t minimises ||x - x*||_H over x_0 + K_t(H_S^{-1} H, H_S^{-1} r_0).
    A, b, nu, lam = _tiny(n=64, d=10, nu=0.05, seed=1, lam=1 + np.arange(10) / 5)
    m, seed = 6, 9
    o = solvers.Options(m_init=m, adaptive=False, stop="fixed", max_iter=t, seed=seed)
    x, _ = solvers.adaptive_pcg(A, b, nu, lam, o)
    H = _H(A, nu, lam)
    HS = SketchedHessian(sk.srht(A, m, seed, 0), nu, lam).matrix()
    xs = np.linalg.solve(H, b)
    M = np.linalg.solve(HS, H)
    v = np.linalg.solve(HS, b)  # x_0 = 0 -> r_0 = b
    K = np.stack([np.linalg.matrix_power(M, j) @ v for j in range(t)], axis=1)
    Q, _ = np.linalg.qr(K)
    c = np.linalg.solve(Q.T @ H @ Q, Q.T @ H @ xs)
    xbest = Q @ c
    assert reference.rel_error(x, xbest) < 1e-7


def test_ihs_error_recursion():
    # Proof of Theorem "rate IHS": x_{t+1} - x* = (I - mu H_S^{-1} H)(x_t - x*), mu = 1 - rho.
    A, b, nu, lam = _tiny(n=64, d=8, nu=0.2, seed=2)
    rho, m, seed = 0.2, 16, 4
    H = _H(A, nu, lam)
    HS = SketchedHessian(sk.srht(A, m, seed, 0), nu, lam).matrix()
    xs = np.linalg.solve(H, b)
    T = np.eye(8) - (1 - rho) * np.linalg.solve(HS, H)
    e = -xs
    for t in range(1, 5):
        o = solvers.Options(method="ihs", rho=rho, m_init=m, adaptive=False, stop="fixed", max_iter=t, seed=seed)
        x, _ = solvers.adaptive_ihs(A, b, nu, lam, o)
        e = T @ e
        np.testing.assert_allclose(x - xs, e, rtol=1e-8, atol=1e-11)


def test_ihs_one_step_full_sketch_contracts_by_rho():
    # With H_S = H the IHS error after one step is exactly rho (x_0 - x*) (mu = 1 - rho).
    A, b, nu, lam = _tiny(n=30, d=5)
    rho = 0.3
    o = solvers.Options(method="ihs", rho=rho, m_init=32, adaptive=False, stop="fixed", max_iter=1)
    x, _ = solvers.adaptive_ihs(A, b, nu, lam, o)
    xs = np.linalg.solve(_H(A, nu, lam), b)
    np.testing.assert_allclose(x - xs, rho * (0 - xs), rtol=1e-10, atol=1e-13)


def test_decrement_bracket():
    # Proof of the decrement lemma: delta/lambda_max(C_S) <= delta~ <= delta/lambda_min(C_S).
    A, b, nu, lam = _tiny(n=128, d=9, nu=0.05, seed=5)
    H = _H(A, nu, lam)
    xs = np.linalg.solve(H, b)
    P = SketchedHessian(sk.srht(A, 12, 2, 0), nu, lam)
    w, V = np.linalg.eigh(H)
    Hh = V @ np.diag(w ** -0.5) @ V.T
    cs = np.linalg.eigvalsh(Hh @ P.matrix() @ Hh)
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.standard_normal(9)
        g = H @ x - b
        dt = 0.5 * g @ P.apply(g)
        dl = 0.5 * (x - xs) @ H @ (x - xs)
        assert dl / cs.max() * (1 - 1e-10) <= dt <= dl / cs.min() * (1 + 1e-10)


@pytest.fixture(scope="module")
def small():
    P = synth.make_workload("pcg_n4096_d256", seed=0)
    P["xref"] = reference.reference_solution(P["A"], P["b"], P["nu"], P["lam"])
    return P


@pytest.mark.parametrize("method", ["pcg", "ihs", "polyak"])
@pytest.mark.parametrize("kind", ["srht", "gauss", "sjlt", "srht_reuse", "srht_nested"])
def test_solution_accuracy(small, method, kind):
    o = solvers.Options(method=method, sketch=kind, m_init=8, tol=1e-10, seed=1)
    x, info = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], o)
    assert info.status == "ok"
    assert reference.rel_error(x, small["xref"]) <= 1e-10
    assert info.final_m <= sk.padded_size(4096)


def test_adaptive_invariants(small):
    o = solvers.Options(m_init=8, seed=2)
    x, info = solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"], o)
    tr = info.trace
    ms = [e["m"] for e in tr]
    assert all(m2 >= m1 for m1, m2 in zip(ms, ms[1:]))
    assert all(math.log2(m / 8).is_integer() for m in ms)
    assert info.resketches <= math.ceil(math.log2(4096 / 8))
    for a, b_ in zip(tr, tr[1:]):
        if a["accept"]:
            assert np.max(a["log_ratio"]) <= a["threshold"] or a["m"] == 4096
            assert b_["t"] == a["t"] + 1 and b_["m"] == a["m"]
        else:
            assert np.max(a["log_ratio"]) > a["threshold"]
            assert b_["t"] == a["t"] and b_["m"] == 2 * a["m"]
    # one pass per candidate step plus one explicit residual per rejection at x_t != 0
    rej_nonzero = sum(1 for e in tr if not e["accept"] and e["t"] > 0)
    assert info.a_passes == info.attempts + rej_nonzero


def test_forced_rejection_restarts(small):
    A, b, nu, lam = small["A"], small["b"], small["nu"], small["lam"]
    o = solvers.Options(m_init=1024, seed=2, force_reject_at=(3,))
    x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    t3 = [e for e in info.trace if e["t"] == 3]
    assert not t3[0]["accept"] and t3[1]["m"] == 2048
    assert info.a_passes == info.attempts + 1
    assert reference.rel_error(x, small["xref"]) <= 1e-10


def test_linear_decay_after_last_resize(small):
    # Condition "linear convergence" for PCG (eq. "rate pcg"): once the sketch satisfies the
    # embedding event, delta_t <= 4 phi^(t - T0) delta_T0.
    A, b, nu, lam = small["A"], small["b"], small["nu"], small["lam"]
    o = solvers.Options(m_init=8, seed=1, keep_iterates=True)
    x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    acc = [e for e in info.trace if e["accept"] and "x" in e]
    mfin = info.final_m
    it = [e for e in acc if e["m"] == mfin]
    xs = small["xref"]
    dl = [float(reference.h_norm_error(A, nu, lam, e["x"][:, 0], xs)) for e in it]
    d0 = dl[0]
    # embedding event of the final sketch
    H = _H(A, nu, lam)
    w, V = np.linalg.eigh(H)
    Hh = V @ np.diag(w ** -0.5) @ V.T
    k_last = it[0]["k"]
    HS = SketchedHessian(sk.srht(A, mfin, 1, k_last), nu, lam).matrix()
    dev = np.max(np.abs(np.linalg.eigvalsh(Hh @ HS @ Hh) - 1))
    rho_eff = max(dev ** 2, 1e-6) if dev < 1 else None
    assert rho_eff is not None
    phi, _ = solvers.pcg_constants(rho_eff)
    for j, dj in enumerate(dl):
        if reference.rel_error(it[j]["x"][:, 0], xs) < 1e-12:
            break
        assert dj <= 4 * phi ** j * d0 * (1 + 1e-6)
    # and the decay is geometric: at least 5x per step on average
    n_use = max(2, min(len(dl), 6))
    assert (dl[n_use - 1] / dl[0]) ** (1 / (n_use - 1)) < 0.2


def test_m_tracks_effective_dimension():
    # Adaptivity theorem / Sec. 5: the final sketch size follows d_e (not d) as nu varies.
    res = []
    for i, nu in enumerate((1e-1, 1e-2, 1e-3)):
        P = synth.make_problem(8192, 256, "geo:0.98", nu, seed=40 + i)
        de = reference.effective_dimension_closed(P["sigma"], nu)
        o = solvers.Options(m_init=1, seed=7, tol=1e-8)
        x, info = solvers.adaptive_pcg(P["A"], P["b"], nu, None, o)
        assert info.status == "ok"
        res.append((de, info.final_m))
    des = [r[0] for r in res]
    ms = [r[1] for r in res]
    assert des == sorted(des)
    assert ms == sorted(ms)
    for de, m in res:
        assert m < 8192
        assert 1 <= m / de <= 64


def test_multiple_rhs_and_equivalence(small):
    A, nu, lam = small["A"], small["nu"], small["lam"]
    rng = np.random.default_rng(5)
    B = A.T @ rng.standard_normal((A.shape[0], 3))
    o = solvers.Options(m_init=8, seed=4)
    X, info = solvers.adaptive_pcg(A, B, nu, lam, o)
    Xr = reference.reference_solution(A, B, nu, lam)
    assert np.all(reference.rel_error(X, Xr) <= 1e-10)
    x1, i1 = solvers.adaptive_pcg(A, B[:, 0], nu, lam, o)
    x2, i2 = solvers.adaptive_pcg(A, B[:, :1], nu, lam, o)
    np.testing.assert_array_equal(x1, x2[:, 0])
    assert i1.iterations == i2.iterations and i1.final_m == i2.final_m


def test_stop_rules_and_status(small):
    A, b, nu, lam = small["A"], small["b"], small["nu"], small["lam"]
    for stop in ("dtilde_rel", "remark"):
        o = solvers.Options(m_init=8, seed=1, stop=stop, tol=1e-12 if stop == "remark" else 1e-9)
        x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
        assert info.status == "ok" and info.iterations > 0
    o = solvers.Options(m_init=8, seed=1, stop="fixed", max_iter=5)
    x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    assert info.status == "ok" and info.iterations == 5
    o = solvers.Options(m_init=8, seed=1, max_iter=3)
    x, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    assert info.status == "max_iter" and info.iterations == 3
    x, info = solvers.adaptive_pcg(A, np.zeros(A.shape[1]), nu, lam, solvers.Options(m_init=8))
    assert info.iterations == 0 and not np.any(x)


def test_validation():
    A, b, nu, lam = _tiny()
    for kw, args in [({}, (A, b, 0.0, lam)), ({}, (A, b, nu, -lam)), ({"rho": 1.0}, (A, b, nu, lam)),
                     ({"m_init": 0}, (A, b, nu, lam))]:
        with pytest.raises(ValueError):
            solvers.adaptive_pcg(*args, solvers.Options(**kw))


def _spd_problem(n, d, seed, decay=0.7, nu=0.3):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = (U * decay ** np.arange(d)) @ V.T
    lam = 1 + rng.random(d)
    b = rng.standard_normal(d)
    return A, b, nu, lam


def test_cg_terminates_in_d_steps():
    # in exact arithmetic CG on a d x d SPD system reaches x* after at most d steps
    A, b, nu, lam = _spd_problem(40, 6, 1)
    H = A.T @ A + nu ** 2 * np.diag(lam)
    xs = np.linalg.solve(H, b)
    x, info = solvers.cg(A, b, nu, lam, solvers.Options(stop="fixed", max_iter=6))
    assert info.iterations == 6 and info.a_passes == 6
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_cg_krylov_optimality():
    # x_t minimises the H-norm error over x_0 + span{r_0, H r_0, ..., H^{t-1} r_0}
    A, b, nu, lam = _spd_problem(60, 9, 2, decay=0.8)
    H = A.T @ A + nu ** 2 * np.diag(lam)
    xs = np.linalg.solve(H, b)
    x0 = np.random.default_rng(3).standard_normal(9)
    r0 = b - H @ x0
    w, V = np.linalg.eigh(H)
    Hh = V @ np.diag(np.sqrt(w)) @ V.T
    for t in range(1, 5):
        K = np.stack([np.linalg.matrix_power(H, j) @ r0 for j in range(t)], axis=1)
        coef, *_ = np.linalg.lstsq(Hh @ K, Hh @ (xs - x0), rcond=None)
        best = x0 + K @ coef
        x, _ = solvers.cg(A, b, nu, lam, solvers.Options(stop="fixed", max_iter=t, x0=x0))
        assert np.linalg.norm(Hh @ (x - best)) <= 1e-9 * np.linalg.norm(Hh @ (xs - x0))


def test_cg_xrel_bounds_the_error(small):
    o = solvers.Options(method="cg", tol=1e-8, max_iter=5000)
    x, info = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], o)
    assert info.status == "ok" and info.final_m == 0
    assert reference.rel_error(x, small["xref"]) <= 1e-8
    assert info.a_passes == info.iterations == len(info.trace)
    with pytest.raises(ValueError):
        solvers.cg(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(stop="remark"))


def test_rho_outside_the_guarantee_warns(small):
    o = solvers.Options(rho=0.3, m_init=8, max_iter=2, stop="fixed")
    with pytest.warns(UserWarning, match="rho >= 1/4"):
        solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"], o)


@pytest.mark.parametrize("n,d,c,with_lam", [(40, 1500, 1, True), (64, 3000, 3, True), (48, 200, 2, False)])
def test_dual_form_matches_the_primal_solution(n, d, c, with_lam):
    # The dual route (eq. "dual optimization problem") must land on the primal x* = H^{-1} b,
    # computed here by the refined direct solve of the primal: a wrong sign or a dropped
    # Lambda in the map back, or a wrong dual right-hand side, fails this.
    rng = np.random.default_rng(n + d)
    A = rng.standard_normal((n, d)) / math.sqrt(d) * (0.9 ** np.arange(n))[:, None]
    lam = 1.0 + rng.random(d) if with_lam else None
    b = rng.standard_normal((d, c))
    nu = 0.05
    x, w, info = solvers.dual_solve(A, b, nu, lam, solvers.Options(tol=1e-12))
    assert info.status == "ok"
    xr = reference.reference_solution(A, b, nu, lam)
    assert np.max(reference.rel_error(x, xr)) <= 1e-10
    # at the solution the dual variable is A x*
    assert np.linalg.norm(A @ x - w) <= 1e-9 * np.linalg.norm(w)
    # the dual problem has n unknowns: the sketch never exceeds the padded size of its d rows
    assert info.final_m <= 1 << (d - 1).bit_length()


def test_dual_form_vector_rhs_and_validation():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((16, 300))
    b = rng.standard_normal(300)
    x, w, _ = solvers.dual_solve(A, b, 1.0, None, solvers.Options(tol=1e-12))
    assert x.shape == (300,) and w.shape == (16,)
    assert np.linalg.norm(x - reference.direct_solve(A, b, 1.0)) <= 1e-10 * np.linalg.norm(x)
    with pytest.raises(ValueError):
        solvers.dual_solve(A, b, 1.0, None, solvers.Options(x0=np.zeros(16)))
    with pytest.raises(ValueError):
        solvers.dual_solve(A, b[:10], 1.0)


def _golden_polyak_table():
    import os

    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "polyak_bound_table.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append((float(f[0]), f[1], f[2], len(f) > 3 and f[3] == "exp_typo"))
    return rows


def test_polyak_bound_matches_the_printed_table():
    # The paper's table of (alpha(t, rho) beta_rho^omega(t))^(1/t) (heavy-ball appendix): every
    # entry within one unit of its last printed digit (two entries after the exponent reading).
    rows = _golden_polyak_table()
    assert len(rows) == 28
    for rho, t, txt, typo in rows:
        mant, _, ex = txt.partition("e")
        digits = len(mant.split(".")[1]) if "." in mant else 0
        unit = 10.0 ** ((int(ex) if ex else 0) - digits)
        printed = float(txt)
        if typo:
            printed, unit = printed / 10.0, unit / 10.0
        if t == "inf":
            v = solvers.polyak_constants(rho)[1]
        else:
            v = math.exp(solvers.polyak_log_bound(int(t), rho) / int(t))
        assert abs(v - printed) <= unit, (rho, t, v, txt)


@pytest.mark.parametrize("rho", [0.3, 0.125, 0.01])
def test_polyak_constants_are_the_heavy_ball_lemma_choice(rho):
    # mu_rho, beta_rho of the corollary are the lemma's mu = 4/(sqrt(l)+sqrt(L))^2 and
    # beta = ((sqrt(L)-sqrt(l))/(sqrt(L)+sqrt(l)))^2 for the spectrum of C_S^{-1} in
    # [1/(1+sqrt rho), 1/(1-sqrt rho)]
    lo, hi = 1.0 / (1.0 + math.sqrt(rho)), 1.0 / (1.0 - math.sqrt(rho))
    mu, beta = solvers.polyak_constants(rho)
    assert mu == pytest.approx(4.0 / (math.sqrt(lo) + math.sqrt(hi)) ** 2, rel=1e-13)
    assert beta == pytest.approx(((math.sqrt(hi) - math.sqrt(lo)) / (math.sqrt(hi) + math.sqrt(lo))) ** 2, rel=1e-12)


def test_polyak_error_recursion():
    # Heavy-ball appendix: x_{t+1} - x* = (I - mu H_S^{-1} H)(x_t - x*) + beta (x_t - x_{t-1}),
    # starting with x_{-1} = x_0 = 0.
    A, b, nu, lam = _tiny(n=64, d=8, nu=0.2, seed=2)
    rho, m, seed = 0.2, 16, 4
    mu, beta = solvers.polyak_constants(rho)
    H = _H(A, nu, lam)
    HS = SketchedHessian(sk.srht(A, m, seed, 0), nu, lam).matrix()
    xs = np.linalg.solve(H, b)
    T = np.eye(8) - mu * np.linalg.solve(HS, H)
    e_prev = e = -xs
    for t in range(1, 6):
        o = solvers.Options(method="polyak", rho=rho, m_init=m, adaptive=False, stop="fixed", max_iter=t, seed=seed)
        x, _ = solvers.adaptive_ihs(A, b, nu, lam, o)
        e, e_prev = T @ e + beta * (e - e_prev), e
        np.testing.assert_allclose(x - xs, e, rtol=1e-8, atol=1e-11)


def test_polyak_resize_restarts_the_momentum(small):
    # a rejection at t = 3 (forced) restarts at x_3 with x_prev = x_3: the accepted step that
    # follows is a plain step of size mu_rho (no momentum term) with the new sketch
    o = solvers.Options(method="polyak", m_init=64, seed=3, stop="fixed", max_iter=4, force_reject_at=(3,),
                        keep_iterates=True)
    x, info = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], o)
    acc = [e for e in info.trace if e["accept"]]
    last = info.trace[-1]
    assert last["accept"] and last["t"] == 3 and not info.trace[-2]["accept"] and info.trace[-2]["t"] == 3
    x3 = acc[2]["x"][:, 0]
    mu, _ = solvers.polyak_constants(o.rho)
    HS = SketchedHessian(sk.srht(small["A"], last["m"], 3, last["k"]), small["nu"], small["lam"])
    g3 = solvers.hess_apply(small["A"], small["nu"], small["lam"], x3[:, None])[:, 0] - small["b"]
    np.testing.assert_allclose(x, x3 - mu * HS.apply(g3[:, None])[:, 0], rtol=1e-9, atol=1e-12)
