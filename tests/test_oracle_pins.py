"""Pins of the oracle's constants, improvement test and stop rules against values evaluated by hand
from the paper's definitions, and against decisions recomputed here from stored iterates.

* Algorithm 2 sets phi(rho) = (1 - sqrt(1-rho)) / (1 + sqrt(1-rho)) and c(rho) = 4 (1+sqrt rho)/(1-sqrt rho);
  the notation section defines c(alpha, rho) = alpha (1+sqrt rho)/(1-sqrt rho); Theorem "rate IHS" gives
  the IHS phi = rho, alpha = 1 and the step mu = 1 - rho; the heavy-ball corollary gives mu_rho and beta_rho.
  The literals below were evaluated with 30-digit decimal arithmetic (sqrt(7/8) = 0.93541434669348534...,
  sqrt(1/8) = 0.35355339059327376..., sqrt(0.7) = 0.83666002653407554..., sqrt(0.3) = 0.54772255750516611...).
* The improvement test of Algorithms 1 and 2 compares D+/D_I with c phi^(t+1-I).  The replay below forms
  H_S = (SA)^T SA + nu^2 Lambda densely from the sketch of each attempt, recomputes every decrement from the
  stored candidate and restart iterates with explicit residuals, and decides each attempt with the exponent
  t+1-I; it must reproduce every accept/reject decision of the oracle, and the plausible alternative
  exponents (t-I, t+1, t+2-I) must not.
* The Remark on termination stops at 1/2 D_t <= eps / (m_delta + 1) with m_delta of the SRHT concentration
  theorem (16 log(16 d_e/delta) (sqrt d_e + sqrt(8 log(2n/delta)))^2) at d_e := d, delta = 1/d.
* The relative-decrement rule stops at D_t / D_0 <= tol^2.
"""
import math

import numpy as np
import pytest

from oracle import sketch as sk
from oracle import solvers

# rho = 1/8 and rho = 0.3 (hand-evaluated, 30-digit decimal arithmetic)
PCG = {0.125: (0.0333704529042344576650050707339, 8.37534528542421725440385994103),
       0.3: (0.0889331564394963468121864947658, 13.6882578000590412966510832320)}
IHS = {0.125: (0.125, 2.09383632135605431360096498526, 0.875),
       0.3: (0.3, 3.42206445001476032416277080800, 0.7)}
POLYAK = {0.125: (0.904199146291205150456879436892, 0.0333704529042344576650050707339),
          0.3: (0.762253209507647442768530546338, 0.0889331564394963468121864947658)}
# m_delta of the SRHT theorem with d_e := d and delta = 1/d
M_DELTA = {(4096, 256): 159205.425142347609886215447526}


@pytest.mark.parametrize("rho", [0.125, 0.3])
def test_constants_hand_evaluated(rho):
    phi, c = solvers.pcg_constants(rho)
    assert phi == pytest.approx(PCG[rho][0], rel=1e-13)
    assert c == pytest.approx(PCG[rho][1], rel=1e-13)
    phi_i, c_i, mu = solvers.ihs_constants(rho)
    assert phi_i == pytest.approx(IHS[rho][0], rel=1e-15)
    assert c_i == pytest.approx(IHS[rho][1], rel=1e-13)
    assert mu == pytest.approx(IHS[rho][2], rel=1e-15)
    mu_p, beta = solvers.polyak_constants(rho)
    assert mu_p == pytest.approx(POLYAK[rho][0], rel=1e-13)
    assert beta == pytest.approx(POLYAK[rho][1], rel=1e-13)


def test_constants_reject_plausible_slips():
    # the literals themselves tell the paper's c apart from (1+rho)/(1-rho) and from a dropped factor 4
    phi, c = PCG[0.125]
    assert abs(c - 4 * 1.125 / 0.875) > 1.0 and abs(c - c / 4) > 1.0
    assert abs(IHS[0.125][1] - 1.125 / 0.875) > 0.5


def test_remark_m_delta_hand_evaluated():
    assert solvers.remark_m_delta(4096, 256) == pytest.approx(M_DELTA[(4096, 256)], rel=1e-12)


def _problem(n=256, d=16, nu=0.05, seed=11):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = (U * (0.7 ** np.arange(d))) @ V.T
    lam = 1 + rng.random(d)
    b = A.T @ rng.standard_normal(n)
    return A, b, nu, lam


class _Dense:
    """Decrements formed densely from the sketch of an attempt (no use of the oracle's factorisation)."""

    def __init__(self, A, b, nu, lam, seed, ihs):
        self.A, self.b, self.nu, self.lam, self.seed, self.ihs = A, b, nu, lam, seed, ihs
        self.H = A.T @ A + nu ** 2 * np.diag(lam)
        self._hs = {}

    def hs(self, m, k):
        if (m, k) not in self._hs:
            SA = sk.srht(self.A, m, self.seed, k)
            self._hs[(m, k)] = SA.T @ SA + self.nu ** 2 * np.diag(self.lam)
        return self._hs[(m, k)]

    def dec(self, x, m, k):
        r = self.b - self.H @ np.ravel(x)
        D = float(r @ np.linalg.solve(self.hs(m, k), r))
        return 0.5 * D if self.ihs else D


def _replay(trace, dense, log_c, log_phi, exponent, m_cap):
    """Accept/reject decisions of the improvement test recomputed from the stored iterates."""
    I, xI, xt = 0, np.zeros(dense.A.shape[1]), np.zeros(dense.A.shape[1])
    out = []
    for e in trace:
        t, m, k = e["t"], e["m"], e["k"]
        lr = math.log(dense.dec(e["xp"], m, k) / dense.dec(xI, m, k))
        thr = log_c + exponent(t, I) * log_phi
        acc = lr <= thr or m >= m_cap
        out.append((acc, abs(lr - thr)))
        if acc:
            xt = np.ravel(e["xp"]).copy()
        else:
            I, xI = t, xt.copy()
    return out


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_improvement_test_exponent_from_iterates(method):
    A, b, nu, lam = _problem()
    o = solvers.Options(method=method, m_init=1, seed=5, keep_iterates=True, tol=1e-12)
    _, info = solvers.solve(A, b, nu, lam, o)
    tr = info.trace
    if method == "pcg":
        phi, c = PCG[0.125]
    else:
        phi, c = IHS[0.125][:2]
    dense = _Dense(A, b, nu, lam, 5, ihs=method == "ihs")
    m_cap = sk.padded_size(A.shape[0])
    exps = {"t+1-I": lambda t, I: t + 1 - I, "t-I": lambda t, I: t - I, "t+1": lambda t, I: t + 1,
            "t+2-I": lambda t, I: t + 2 - I}
    got = {name: _replay(tr, dense, math.log(c), math.log(phi), f, m_cap) for name, f in exps.items()}
    oracle = [e["accept"] for e in tr]
    # the scenario exercises restarts at I > 0 followed by accepted runs of several steps
    assert sum(1 for e in tr if not e["accept"]) >= 4
    assert max(e["t"] for e in tr) >= 8
    for (acc, margin), want in zip(got["t+1-I"], oracle):
        if margin > 1e-8:
            assert acc == want
    for name in ("t-I", "t+1", "t+2-I"):
        assert [a for a, _ in got[name]] != oracle, name


def test_dtilde_rel_stops_at_tol_squared():
    A, b, nu, lam = _problem()
    dense = _Dense(A, b, nu, lam, 5, ihs=False)
    o = solvers.Options(m_init=16, seed=5, keep_iterates=True, stop="fixed", max_iter=10)
    _, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    acc = [e for e in info.trace if e["accept"]]
    D0 = dense.dec(np.zeros(A.shape[1]), info.trace[0]["m"], info.trace[0]["k"])
    ratios = [dense.dec(e["x"], e["m"], e["k"]) / D0 for e in acc]
    tol = 10 ** (0.5 * math.log10(math.sqrt(ratios[5] * ratios[6])))  # tol^2 between steps 6 and 7
    want = next(i + 1 for i, r in enumerate(ratios) if r <= tol ** 2)
    slip = next(i + 1 for i, r in enumerate(ratios) if r <= tol)
    assert want == 7 and slip < want
    o2 = solvers.Options(m_init=16, seed=5, stop="dtilde_rel", tol=tol)
    _, info2 = solvers.adaptive_pcg(A, b, nu, lam, o2)
    assert info2.status == "ok" and info2.iterations == want


def test_remark_rule_stops_at_half_decrement():
    A, b, nu, lam = _problem()
    n, d = A.shape
    dense = _Dense(A, b, nu, lam, 5, ihs=False)
    o = solvers.Options(m_init=16, seed=5, keep_iterates=True, stop="fixed", max_iter=10)
    _, info = solvers.adaptive_pcg(A, b, nu, lam, o)
    acc = [e for e in info.trace if e["accept"]]
    D = [dense.dec(e["x"], e["m"], e["k"]) for e in acc]
    # m_delta at n = 256, d = 16 (hand-evaluated like M_DELTA): 16 log(4096) (4 + sqrt(8 log 8192))^2
    m_delta = 16 * math.log(4096.0) * (4.0 + math.sqrt(8 * math.log(8192.0))) ** 2
    assert solvers.remark_m_delta(n, d) == pytest.approx(m_delta, rel=1e-14)
    assert m_delta == pytest.approx(20762.5686349, rel=1e-10)
    # eps so that 1/2 D_5 <= eps/(m_delta+1) < D_5 and 1/2 D_4 > eps/(m_delta+1)
    eps = 0.75 * D[4] * (m_delta + 1.0)
    assert 0.5 * D[3] > 0.75 * D[4] and D[5] <= 0.75 * D[4]
    o2 = solvers.Options(m_init=16, seed=5, stop="remark", tol=eps)
    _, info2 = solvers.adaptive_pcg(A, b, nu, lam, o2)
    assert info2.status == "ok" and info2.iterations == 5
