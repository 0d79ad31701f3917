"""Adaptive sketch-size PCG and IHS, written from the paper's algorithms.  Test infrastructure.

Problem (eq. "main optimization problem"): minimise f(x) = 1/2 x^T H x - b^T x with
H = A^T A + nu^2 Lambda, A in R^{n x d}, Lambda diagonal.

* ``adaptive_pcg`` follows Algorithm 2 (adaptive PCG): PCG steps (eq. "pcg update") with
  preconditioner H_S; after each candidate step the approximate Newton decrement ratio is
  compared with c(rho) * phi(rho)^(t+1-I), phi = (1-sqrt(1-rho))/(1+sqrt(1-rho)),
  c = 4 (1+sqrt rho)/(1-sqrt rho); on failure I <- t, m <- 2m, a fresh S is drawn, H_S is
  refactored and the residual r_t = b - H x_t is recomputed explicitly.
* ``adaptive_ihs`` follows Algorithm 1 with the IHS update (eq. "ihs") and the constants of
  Theorem "rate IHS": step mu = 1 - rho, phi = rho, alpha = 1, so c = (1+sqrt rho)/(1-sqrt rho);
  its decrement carries the 1/2 of Sec. 2.3.  A rejection needs no pass over A: the gradient
  at x_t is unchanged.

Readings where the paper is silent (each also listed in the design notes):
  * test in the log domain; equality passes (the paper rejects on ">"); a candidate with
    decrement <= 0 passes;
  * m is capped at n' (the padded Hadamard size) for both embeddings; at the cap a failed test
    is accepted and ``m_cap_reached`` is set;
  * x_0 = 0 gives r_0 = b (-b for the IHS gradient) without a pass over A, and so does a
    restart at x_t = 0;
  * stop rules (the paper prescribes none, Sec. 1.3 and the Remark on termination):
      'xrel'       (default) (1+sqrt rho) * D <= nu^2 min(lambda) tol^2 ||x_t||^2 with D the
                   decrement r^T H_S^{-1} r (= 2 x the 1/2-weighted decrement); from the
                   decrement lemma, delta <= (1+sqrt rho) * delta~ under the embedding event,
                   and delta >= 1/2 nu^2 min(lambda) ||x - x*||^2;
      'dtilde_rel' D_t / D_0 <= tol^2;
      'fixed'      exactly max_iter accepted steps (the algorithms' iteration number T);
      'remark'     delta~_t <= tol / (m_delta + 1), m_delta from the SRHT concentration
                   theorem with d_e replaced by d and failure probability 1/d;
    always: stop a column when its decrement or residual is exactly zero;
  * matrix variables (c right-hand sides, Sec. 5 "accounts for matrix variables"): the
    columns share S and H_S; a candidate step is rejected if any active column fails the
    test; on rejection every active column restarts at its own x_t; a column that meets the
    stop rule is frozen.  With c = 1 this is exactly Algorithm 2 / Algorithm 1.
  * ``max_iter`` bounds the number of accepted steps t (the loop "while t < T").

``cg`` is the paper's unpreconditioned conjugate-gradient baseline (Sec. 5).
``dual_solve`` takes the dual route of Sec. 1 for n < d (eq. "dual optimization problem").
Method 'polyak' of ``adaptive_ihs`` is the heavy-ball (Polyak-IHS) update of the appendix
"Heavy-ball Acceleration and Adaptivity" with the corollary's mu_rho, beta_rho and, for the
adaptive form, its finite-time factor alpha(t, rho) beta_rho^omega(t) in the test (the paper
describes this adaptive version but calls it impractical; readings in ``adaptive_ihs``).

Pins (tests/test_oracle_solvers.py): one-step convergence when m = n' (H_S = H); Krylov
optimality of PCG (Theorem "rate cg") by brute-force least squares on tiny problems; the IHS
error recursion (proof of Theorem "rate IHS"); the decrement bracket (proof of the decrement
lemma); invariants of the adaptive control (accepted steps satisfy the test, m doubles, K
bounded, forced rejections recompute r_t = b - H x_t); rel. error <= 1e-10 against the
refined direct solution; for ``cg``: termination in d steps, Krylov optimality in the
H-norm by brute-force least squares, and the xrel bound on the true error; for
``dual_solve``: the primal x* of the refined direct solve and A x* = w*; for 'polyak': the
paper's printed table of the finite-time factor (tests/golden/polyak_bound_table.txt), mu_rho
and beta_rho as the heavy-ball lemma's choice, the heavy-ball error recursion, the momentum
restart at a resize.
"""
import math
import warnings
from dataclasses import dataclass, field

import numpy as np

from . import sketch as sk
from .factor import NotSPDError, SketchedHessian


@dataclass
class Options:
    method: str = "pcg"          # 'pcg' | 'ihs' | 'polyak' (heavy-ball IHS) | 'cg' (unpreconditioned baseline)
    sketch: str = "srht"         # 'srht' | 'gauss' | 'sjlt' | 'srht_reuse' | 'srht_nested' (variants)
    rho: float = 0.125
    m_init: int = 1
    m_max: int = 0               # 0 -> n'
    max_iter: int = 200
    stop: str = "xrel"           # 'xrel' | 'dtilde_rel' | 'fixed' | 'remark'
    tol: float = 1e-10
    seed: int = 0
    problem: int = 0
    adaptive: bool = True
    force_reject_at: tuple = ()  # values of t at which the first candidate step is rejected
    x0: object = None
    keep_iterates: bool = False  # store each candidate (xp) and committed x in the trace (tests)


@dataclass
class Info:
    status: str = "ok"           # 'ok' | 'max_iter' | 'not_spd' | 'nonfinite'
    iterations: int = 0          # accepted steps t
    attempts: int = 0            # candidate steps (accepted + rejected)
    final_m: int = 0
    resketches: int = 0
    a_passes: int = 0            # passes over A (H.v products and explicit residuals)
    m_cap_reached: bool = False
    dtilde_final: object = None
    trace: list = field(default_factory=list)


def pcg_constants(rho):
    """(phi, c) of Algorithm 2."""
    s = math.sqrt(1.0 - rho)
    phi = (1.0 - s) / (1.0 + s)
    c = 4.0 * (1.0 + math.sqrt(rho)) / (1.0 - math.sqrt(rho))
    return phi, c


def ihs_constants(rho):
    """(phi, c, mu) for the IHS: phi = rho, alpha = 1, mu = 1 - rho (Theorem "rate IHS")."""
    c = (1.0 + math.sqrt(rho)) / (1.0 - math.sqrt(rho))
    return rho, c, 1.0 - rho


def polyak_constants(rho):
    """(mu_rho, beta_rho) of the Polyak-IHS corollary (heavy-ball appendix):
    mu = 2 (1 - rho) / (1 + sqrt(1 - rho)), beta = (1 - sqrt(1 - rho)) / (1 + sqrt(1 - rho))."""
    q = math.sqrt(1.0 - rho)
    return 2.0 * (1.0 - rho) / (1.0 + q), (1.0 - q) / (1.0 + q)


def polyak_log_bound(t, rho):
    """log of alpha(t, rho) * beta_rho^omega(t), the finite-time factor of the Polyak-IHS
    corollary: nu(t) = log2(t) + 1 (real-valued), omega(t) = t - 2 nu(t),
    alpha(t, rho) = 3^(nu (nu + 1)) (1 + 4 beta + beta^2)^(2 nu).  t >= 1."""
    _, beta = polyak_constants(rho)
    nu_t = math.log(t) / math.log(2.0) + 1.0
    log_alpha = nu_t * (nu_t + 1.0) * math.log(3.0) + 2.0 * nu_t * math.log(1.0 + 4.0 * beta + beta * beta)
    return log_alpha + (t - 2.0 * nu_t) * math.log(beta)


def remark_m_delta(n, d, delta=None):
    """m_delta of the SRHT concentration theorem with d_e := d (Remark on termination)."""
    de = float(d)
    delta = 1.0 / d if delta is None else delta
    return 16.0 * math.log(16.0 * de / delta) * (math.sqrt(de) + math.sqrt(8.0 * math.log(2.0 * n / delta))) ** 2


def hess_apply(A, nu, lam, P):
    """H P = A^T (A P) + nu^2 Lambda P."""
    return A.T @ (A @ P) + (nu ** 2) * lam[:, None] * P


def _validate(A, b, nu, lam, o):
    n, d = A.shape
    if n < 1 or d < 1:
        raise ValueError("n and d must be >= 1")
    if b.shape[0] != d:
        raise ValueError("b must have d rows")
    if not (np.isfinite(nu) and nu > 0):
        raise ValueError("nu must be finite and > 0")
    if np.any(~np.isfinite(lam)) or np.any(lam <= 0):
        raise ValueError("Lambda must have finite positive entries")
    if not 0.0 < o.rho < 1.0:
        raise ValueError("rho must lie in (0, 1)")
    if o.rho >= 0.25 and o.adaptive:
        # the adaptive methods are defined for rho in (0, 1); their guarantee (Theorem
        # "adaptive") is stated for rho < 1/4
        warnings.warn("rho >= 1/4: outside the range of the adaptive guarantee", stacklevel=3)
    if o.m_init < 1:
        raise ValueError("m_init must be >= 1")
    if o.tol <= 0 and o.stop != "fixed":
        raise ValueError("tol must be > 0")
    if o.method not in ("pcg", "ihs", "polyak"):
        raise ValueError("method must be 'pcg', 'ihs' or 'polyak'")


class _Stopper:
    """Stop rules, evaluated per column after initialisation and after each accepted step."""

    def __init__(self, o, n, d, nu, lam, half):
        self.o = o
        self.scale = (nu ** 2) * float(np.min(lam)) * o.tol ** 2
        self.sr = 1.0 + math.sqrt(o.rho)
        self.half = half  # True when the stored decrement carries the 1/2 (IHS)
        self.D0 = None
        if o.stop == "remark":
            self.remark_thr = o.tol / (remark_m_delta(n, d) + 1.0)

    def full_decrement(self, dt):
        return 2.0 * dt if self.half else dt

    def done(self, dt, x, resid, t, J=None):
        """Boolean per column (J: the column indices dt, x, resid belong to)."""
        D = self.full_decrement(dt)
        if self.D0 is None:
            self.D0 = D.copy()
        D0 = self.D0 if J is None else self.D0[J]
        exact = (dt <= 0) | ~np.any(resid != 0, axis=0)
        s = self.o.stop
        if s == "xrel":
            rule = self.sr * D <= self.scale * np.sum(x * x, axis=0)
        elif s == "dtilde_rel":
            rule = D <= (self.o.tol ** 2) * D0
        elif s == "fixed":
            rule = np.full(D.shape, t >= self.o.max_iter)
        elif s == "remark":
            rule = 0.5 * D <= self.remark_thr
        else:
            raise ValueError(f"unknown stop rule {s!r}")
        return exact | rule


def _as2d(b):
    b = np.asarray(b, dtype=np.float64)
    return (b[:, None], True) if b.ndim == 1 else (b, False)


def _sketch_factor(A, m, o, k, nu, lam):
    SA = sk.sketch(A, m, o.sketch, o.seed, k, o.problem)
    return SketchedHessian(SA, nu, lam)


def adaptive_pcg(A, b, nu, lam=None, opts=None):
    """Adaptive PCG (Algorithm 2).  Returns (x, Info); x has the shape of b."""
    o = opts or Options()
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    B, squeeze = _as2d(b)
    c = B.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    _validate(A, B, nu, lam, o)
    info = Info()
    phi, cc = pcg_constants(o.rho)
    log_phi, log_c = math.log(phi), math.log(cc)
    m_cap = sk.max_sketch_size(n, o.sketch) if o.m_max <= 0 else min(o.m_max, sk.max_sketch_size(n, o.sketch))
    m = min(o.m_init, m_cap)
    k = 0
    try:
        P = _sketch_factor(A, m, o, k, nu, lam)
    except NotSPDError:
        info.status = "not_spd"
        return (np.zeros(d) if squeeze else np.zeros((d, c))), info

    X = np.zeros((d, c)) if o.x0 is None else np.array(o.x0, dtype=np.float64).reshape(d, c)
    if np.any(X != 0):
        R = B - hess_apply(A, nu, lam, X)
        info.a_passes += 1
    else:
        R = B.copy()
    Rt = P.apply(R)
    Pd = Rt.copy()
    Dt = np.sum(R * Rt, axis=0)
    DI = Dt.copy()
    I = t = 0
    stopper = _Stopper(o, n, d, nu, lam, half=False)
    active = ~stopper.done(Dt, X, R, t)
    forced = set()

    while active.any():
        if t >= o.max_iter:
            info.status = "max_iter"
            break
        J = np.flatnonzero(active)
        pJ = Pd[:, J]
        Q = hess_apply(A, nu, lam, pJ)
        info.a_passes += 1
        pHp = np.sum(pJ * Q, axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            alpha = Dt[J] / pHp
        Xp = X[:, J] + alpha * pJ
        Rp = R[:, J] - alpha * Q
        Rtp = P.apply(Rp)
        Dp = np.sum(Rp * Rtp, axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            Pp = Rtp + (Dp / Dt[J]) * pJ
        info.attempts += 1
        if not (np.all(np.isfinite(alpha)) and np.all(np.isfinite(Dp))):
            info.status = "nonfinite"
            break
        thr = log_c + (t + 1 - I) * log_phi
        with np.errstate(divide="ignore"):
            lr = np.where(Dp > 0, np.log(np.maximum(Dp, 1e-300)) - np.log(DI[J]), -np.inf)
        fail = bool(np.any(lr > thr))
        if o.adaptive and t in o.force_reject_at and t not in forced:
            forced.add(t)
            fail = True
        info.trace.append(dict(t=t, m=m, k=k, log_ratio=lr.copy(), threshold=thr, accept=not fail or not o.adaptive or m >= m_cap))
        if o.keep_iterates:
            info.trace[-1]["xp"] = Xp.copy()
        if fail and o.adaptive and m < m_cap:
            I = t
            m = min(2 * m, m_cap)
            k += 1
            info.resketches += 1
            try:
                P = _sketch_factor(A, m, o, k, nu, lam)
            except NotSPDError:
                info.status = "not_spd"
                break
            xJ = X[:, J]
            if np.any(xJ != 0):
                R[:, J] = B[:, J] - hess_apply(A, nu, lam, xJ)
                info.a_passes += 1
            else:
                R[:, J] = B[:, J]
            Rt[:, J] = P.apply(R[:, J])
            Pd[:, J] = Rt[:, J]
            Dt[J] = np.sum(R[:, J] * Rt[:, J], axis=0)
            DI[J] = Dt[J]
            continue
        if fail and o.adaptive:
            info.m_cap_reached = True
        X[:, J], R[:, J], Rt[:, J], Pd[:, J], Dt[J] = Xp, Rp, Rtp, Pp, Dp
        t += 1
        if o.keep_iterates:
            info.trace[-1]["x"] = X.copy()
        active[J] = ~stopper.done(Dt[J], X[:, J], R[:, J], t, J)

    info.iterations = t
    info.final_m = m
    info.dtilde_final = Dt.copy()
    return (X[:, 0] if squeeze else X), info


def adaptive_ihs(A, b, nu, lam=None, opts=None):
    """Adaptive IHS (Algorithm 1 with psi = IHS, mu = 1 - rho).  Returns (x, Info).

    With method 'polyak' the update is the heavy-ball (Polyak-IHS) step of the appendix,
    x+ = x - mu_rho H_S^{-1} g + beta_rho (x - x_prev), with x_prev = x_0 at the start and
    x_prev = x_t after a resize (the momentum restarts with the new sketch), and the test of
    Algorithm 1 takes the corollary's finite-time factor: reject when
    D+/D_I > (1+sqrt rho)/(1-sqrt rho) * alpha(tau, rho) beta_rho^omega(tau), tau = t+1-I.
    """
    o = opts or Options(method="ihs")
    polyak = o.method == "polyak"
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    B, squeeze = _as2d(b)
    c = B.shape[1]
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    _validate(A, B, nu, lam, o)
    info = Info()
    phi, cc, mu = ihs_constants(o.rho)
    beta = 0.0
    if polyak:
        mu, beta = polyak_constants(o.rho)
    log_phi, log_c = math.log(phi), math.log(cc)
    m_cap = sk.max_sketch_size(n, o.sketch) if o.m_max <= 0 else min(o.m_max, sk.max_sketch_size(n, o.sketch))
    m = min(o.m_init, m_cap)
    k = 0
    try:
        P = _sketch_factor(A, m, o, k, nu, lam)
    except NotSPDError:
        info.status = "not_spd"
        return (np.zeros(d) if squeeze else np.zeros((d, c))), info

    X = np.zeros((d, c)) if o.x0 is None else np.array(o.x0, dtype=np.float64).reshape(d, c)
    if np.any(X != 0):
        G = hess_apply(A, nu, lam, X) - B
        info.a_passes += 1
    else:
        G = -B.copy()
    Xprev = X.copy()
    Sd = P.apply(G)
    Dt = 0.5 * np.sum(G * Sd, axis=0)
    DI = Dt.copy()
    I = t = 0
    stopper = _Stopper(o, n, d, nu, lam, half=True)
    active = ~stopper.done(Dt, X, G, t)
    forced = set()

    while active.any():
        if t >= o.max_iter:
            info.status = "max_iter"
            break
        J = np.flatnonzero(active)
        Xp = X[:, J] - mu * Sd[:, J]
        if polyak:
            Xp = Xp + beta * (X[:, J] - Xprev[:, J])
        Gp = hess_apply(A, nu, lam, Xp) - B[:, J]
        info.a_passes += 1
        Sp = P.apply(Gp)
        Dp = 0.5 * np.sum(Gp * Sp, axis=0)
        info.attempts += 1
        if not np.all(np.isfinite(Dp)):
            info.status = "nonfinite"
            break
        thr = log_c + (polyak_log_bound(t + 1 - I, o.rho) if polyak else (t + 1 - I) * log_phi)
        with np.errstate(divide="ignore"):
            lr = np.where(Dp > 0, np.log(np.maximum(Dp, 1e-300)) - np.log(DI[J]), -np.inf)
        fail = bool(np.any(lr > thr))
        if o.adaptive and t in o.force_reject_at and t not in forced:
            forced.add(t)
            fail = True
        info.trace.append(dict(t=t, m=m, k=k, log_ratio=lr.copy(), threshold=thr, accept=not fail or not o.adaptive or m >= m_cap))
        if o.keep_iterates:
            info.trace[-1]["xp"] = Xp.copy()
        if fail and o.adaptive and m < m_cap:
            I = t
            m = min(2 * m, m_cap)
            k += 1
            info.resketches += 1
            try:
                P = _sketch_factor(A, m, o, k, nu, lam)
            except NotSPDError:
                info.status = "not_spd"
                break
            Sd[:, J] = P.apply(G[:, J])
            Dt[J] = 0.5 * np.sum(G[:, J] * Sd[:, J], axis=0)
            DI[J] = Dt[J]
            Xprev[:, J] = X[:, J]
            continue
        if fail and o.adaptive:
            info.m_cap_reached = True
        Xprev[:, J] = X[:, J]
        X[:, J], G[:, J], Sd[:, J], Dt[J] = Xp, Gp, Sp, Dp
        t += 1
        if o.keep_iterates:
            info.trace[-1]["x"] = X.copy()
        active[J] = ~stopper.done(Dt[J], X[:, J], G[:, J], t, J)

    info.iterations = t
    info.final_m = m
    info.dtilde_final = Dt.copy()
    return (X[:, 0] if squeeze else X), info


def cg(A, b, nu, lam=None, opts=None):
    """Unpreconditioned conjugate gradient on H x = b: the baseline of the paper's numerical
    section (Sec. 5), in its textbook (Hestenes-Stiefel) form:

        q = H p,  alpha = r^T r / p^T q,  x += alpha p,  r -= alpha q,
        beta = r+^T r+ / r^T r,  p = r+ + beta p.

    Matrix variables: every column runs its own recurrence; a column that meets the stop rule
    is frozen.  Stop rules (the same names as the adaptive solvers, with the identity in place
    of H_S):
      'xrel'       ||r||^2 <= (nu^2 min(lambda) tol)^2 ||x||^2, which bounds the relative error
                   by tol since ||x - x*|| <= ||H^{-1}|| ||r|| <= ||r|| / (nu^2 min(lambda));
      'dtilde_rel' r^T r <= tol^2 r_0^T r_0;
      'fixed'      exactly max_iter steps;
    and a column with r = 0 stops.  Returns (x, Info) with final_m = 0 (no sketch).
    """
    o = opts or Options()
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    B, squeeze = _as2d(b)
    lam = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    if n < 1 or d < 1 or B.shape[0] != d:
        raise ValueError("bad shapes")
    if not (np.isfinite(nu) and nu > 0):
        raise ValueError("nu must be finite and > 0")
    if o.stop not in ("xrel", "dtilde_rel", "fixed"):
        raise ValueError("CG supports the stop rules 'xrel', 'dtilde_rel' and 'fixed'")
    info = Info()
    c = B.shape[1]
    X = np.zeros((d, c)) if o.x0 is None else np.array(o.x0, dtype=np.float64).reshape(d, c)
    if o.x0 is None:
        R = B.copy()
    else:
        R = B - hess_apply(A, nu, lam, X)
        info.a_passes += 1
    P = R.copy()
    g = np.sum(R * R, axis=0)
    g0 = g.copy()
    scale = (nu ** 2 * float(np.min(lam)) * o.tol) ** 2

    def stopped(gam, Xc, t, J):
        exact = gam <= 0
        if o.stop == "xrel":
            rule = gam <= scale * np.sum(Xc * Xc, axis=0)
        elif o.stop == "dtilde_rel":
            rule = gam <= (o.tol ** 2) * g0[J]
        else:
            rule = np.full(gam.shape, t >= o.max_iter)
        return exact | rule

    active = np.arange(c)
    active = active[~stopped(g, X, 0, active)]
    t = 0
    while active.size and t < o.max_iter:
        J = active
        Q = hess_apply(A, nu, lam, P[:, J])
        info.a_passes += 1
        alpha = g[J] / np.sum(P[:, J] * Q, axis=0)
        X[:, J] += alpha * P[:, J]
        R[:, J] -= alpha * Q
        gn = np.sum(R[:, J] * R[:, J], axis=0)
        P[:, J] = R[:, J] + (gn / g[J]) * P[:, J]
        g[J] = gn
        t += 1
        info.attempts += 1
        info.iterations = t
        info.trace.append({"t": t - 1, "m": 0, "accept": True})
        active = J[~stopped(g[J], X[:, J], t, J)]
    if active.size and o.stop != "fixed":
        info.status = "max_iter"
    return (X[:, 0] if squeeze else X), info


def solve(A, b, nu, lam=None, opts=None):
    o = opts or Options()
    if o.method == "cg":
        return cg(A, b, nu, lam, o)
    return adaptive_ihs(A, b, nu, lam, o) if o.method in ("ihs", "polyak") else adaptive_pcg(A, b, nu, lam, o)


def dual_solve(A, b, nu, lam=None, opts=None):
    """Solve H x = b through the dual problem (eq. "dual optimization problem", Sec. 1): n < d.

    With B = Lambda^{-1/2} A^T (d x n), the dual variable w in R^n minimises
    1/2 w^T (B^T B + nu^2 I_n) w - (A Lambda^{-1} b)^T w: the same problem class with data matrix
    B (d rows, n columns), Lambda = I_n and right-hand side A Lambda^{-1} b, solved here by
    ``solve`` with the options unchanged.  The paper does not write the map back; from the
    primal optimality condition H x* = b one gets x* = Lambda^{-1} (b - A^T w*) / nu^2 (and then
    A x* = w*), computed as Lambda^{-1/2} (Lambda^{-1/2} b - B w) / nu^2.

    Returns (x, w, info); info is the dual solve's (its a_passes count passes over B).  A start
    point is not accepted (opts.x0 must be None).
    """
    o = opts or Options()
    if o.x0 is not None:
        raise ValueError("the dual form takes no start point")
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    b2, squeeze = _as2d(b)
    if b2.shape[0] != d:
        raise ValueError("b must have d rows")
    lam_v = np.ones(d) if lam is None else np.asarray(lam, dtype=np.float64)
    if np.any(~np.isfinite(lam_v)) or np.any(lam_v <= 0):
        raise ValueError("Lambda must have finite positive entries")
    isl = 1.0 / np.sqrt(lam_v)
    Bm = np.ascontiguousarray(A.T * isl[:, None])           # Lambda^{-1/2} A^T, d x n
    bd = A @ (b2 / lam_v[:, None])                           # A Lambda^{-1} b, n x c
    W, info = solve(Bm, bd, nu, None, o)
    W = W.reshape(n, -1)
    X = isl[:, None] * (isl[:, None] * b2 - Bm @ W) / nu ** 2
    return (X[:, 0] if squeeze else X), (W[:, 0] if squeeze else W), info
