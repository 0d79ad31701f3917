"""Solver-level parity of the HIP library against the oracle on small workloads."""
import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
import synth
from oracle import adjoint, reference, solvers

from _helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    P = synth.make_workload("pcg_n4096_d256", seed=0)
    P["xref"] = reference.reference_solution(P["A"], P["b"], P["nu"], P["lam"])
    P["dA"] = to_dev(P["A"])
    P["db"] = to_dev(P["b"])
    P["dlam"] = to_dev(P["lam"])
    return P


def _traj_gpu(info):
    return [(e["t"], e["m"], e["accept"]) for e in info["trace"]]


def _traj_cpu(io):
    return [(e["t"], e["m"], bool(e["accept"])) for e in io.trace]


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_srht_trajectory_and_accuracy(small, method):
    kw = dict(method=method, sketch="srht", m_init=8, seed=1, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["iterations"] == io.iterations and info["final_m"] == io.final_m
    assert info["resketches"] == io.resketches and info["a_passes"] == io.a_passes
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_gaussian_accuracy(small, method):
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], method=method, sketch="gauss",
                        m_init=8, seed=1, tol=1e-10)
    assert info["status"] == "ok"
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert info["final_m"] <= 4096


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_sjlt_trajectory_and_accuracy(small, method):
    kw = dict(method=method, sketch="sjlt", m_init=8, seed=1, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["final_m"] == io.final_m and info["a_passes"] == io.a_passes
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_srht_reuse_trajectory_and_accuracy(small, method):
    kw = dict(method=method, sketch="srht_reuse", m_init=8, seed=1, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["final_m"] == io.final_m and info["a_passes"] == io.a_passes
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9
    # FP64 only
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], sketch="srht_reuse", precision="mixed")


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_srht_nested_trajectory_and_accuracy(small, method):
    # d = 256: the resizes from m = 256 on form the Gram incrementally on the device, the oracle
    # forms it from the whole sketch
    kw = dict(method=method, sketch="srht_nested", m_init=8, seed=1, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["final_m"] == io.final_m and info["a_passes"] == io.a_passes
    assert info["final_m"] >= 1024  # at least two incremental Grams
    # trace series: D after each attempt; within one sketch (same m), accepted attempts'
    # log D differences equal their log-ratio differences (one right-hand side); time stamps grow
    tr = info["trace"]
    assert all(e["dtilde"] > 0 for e in tr)
    assert all(b_["time_ms"] >= a["time_ms"] >= 0 for a, b_ in zip(tr, tr[1:]))
    acc = [e for e in tr if e["accept"]]
    pairs = [(a, b_) for a, b_ in zip(acc, acc[1:]) if a["m"] == b_["m"] and a["t"] + 1 == b_["t"]]
    assert pairs
    for a, b_ in pairs:
        assert np.isclose(np.log(b_["dtilde"] / a["dtilde"]), b_["log_ratio"] - a["log_ratio"], rtol=0, atol=1e-9)
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], sketch="srht_nested", precision="mixed")


def _cholesky_bound(A, nu, lam):
    # forward error of a Cholesky solve of H (and of applying its inverse factors): a small
    # multiple of d kappa(H) u
    H = A.T @ A + nu ** 2 * np.diag(lam)
    return 8 * A.shape[1] * np.linalg.cond(H) * np.finfo(np.float64).eps


def test_direct_baseline_full_size_fixture(small):
    x = aes.solve_direct(small["dA"], small["db"], small["nu"], small["dlam"]).cpu().numpy()
    err = reference.rel_error(x, small["xref"])
    assert err <= _cholesky_bound(small["A"], small["nu"], small["lam"])
    assert err <= 1e-8


@pytest.mark.parametrize("n,d,c,nu", [(1000, 70, 3, 1.0), (5000, 300, 1, 0.5), (777, 130, 32, 0.3),
                                      (100, 300, 2, 0.5)])
def test_direct_baseline_ragged(n, d, c, nu):
    # d = 70: the small-d Gram path and a padded factor (d -> 128); d = 300 and 130: the tiled Gram
    # with ragged tiles; n = 100 < d = 300: H is nu^2 Lambda plus a rank-100 term; 3 and 32
    # right-hand sides, b and x strided
    if n >= d:
        P = synth.make_problem(n, d, "geo:0.99", nu, lam="uniform1_10", nrhs=c, seed=n + d)
        A, lam = P["A"], P["lam"]
        b = P["b"].reshape(d, c)
    else:
        rng = np.random.default_rng(n + d)
        A = rng.standard_normal((n, d)) / np.sqrt(n)
        lam = 1.0 + 9.0 * rng.random(d)
        b = rng.standard_normal((d, c))
    xref = reference.reference_solution(A, b, nu, lam)
    db = torch.zeros((d, c + 2), dtype=torch.float64, device="cuda")
    db[:, :c] = to_dev(b)
    dx = torch.full((d, c + 3), 7.0, dtype=torch.float64, device="cuda")
    aes.solve_direct(to_dev(A), db[:, :c], nu, to_dev(lam), x=dx[:, :c])
    assert np.all(dx[:, c:].cpu().numpy() == 7.0)
    err = reference.rel_error(dx[:, :c].cpu().numpy(), xref)
    assert np.max(err) <= min(1e-11, _cholesky_bound(A, nu, lam))


def test_direct_baseline_rejects_bad_arguments(small):
    dx = torch.full((256,), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve_direct(small["dA"], small["db"], 0.0, small["dlam"], x=dx)
    b33 = torch.zeros((256, 33), dtype=torch.float64, device="cuda")
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve_direct(small["dA"], b33, small["nu"], small["dlam"])
    assert torch.all(dx == 3.0)


@pytest.mark.parametrize("kw,final_m", [(dict(m_init=8, m_max=600), 600), (dict(method="ihs", m_init=8, m_max=600), 600),
                                        (dict(m_init=512), 1024)])
def test_srht_nested_uneven_cap_and_cholesky_start(small, kw, final_m):
    # m_max = 600: the last resize grows 512 -> 600, so the kept Gram enters with weight 512/600;
    # m_init = 512 >= d: the first sketch already takes the Cholesky branch (a full Gram), the
    # next one is incremental
    kw = dict(sketch="srht_nested", seed=1, tol=1e-10, **kw)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["final_m"] == io.final_m == final_m
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("kw", [dict(m_init=8), dict(m_init=512, adaptive=False)])
def test_polyak_trajectory_and_accuracy(small, kw):
    kw = dict(method="polyak", seed=1, tol=1e-10, max_iter=500, **kw)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=512, **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["iterations"] == io.iterations and info["final_m"] == io.final_m
    assert info["a_passes"] == io.a_passes
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("force", [(), (3,)])
def test_polyak_iterates_match_the_oracle(small, force):
    # five accepted heavy-ball steps (with a forced rejection at t = 3: the momentum restart)
    kw = dict(method="polyak", m_init=64, seed=3, stop="fixed", max_iter=5, force_reject_at=force, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=64,
                        **{**kw, "force_reject_at": force[0] if force else -1})
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert _traj_gpu(info) == _traj_cpu(io) and info["iterations"] == 5
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-10


def test_polyak_several_rhs(small):
    rng = np.random.default_rng(8)
    Bm = small["A"].T @ rng.standard_normal((4096, 3))
    X, info = aes.solve(small["dA"], to_dev(Bm), small["nu"], small["dlam"], method="polyak", m_init=512,
                        adaptive=False, seed=2, tol=1e-10)
    Xr = reference.reference_solution(small["A"], Bm, small["nu"], small["lam"])
    assert info["status"] == "ok" and np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)


@pytest.mark.parametrize("precision", ["mixed", "mixed_fp32"])
def test_polyak_mixed_precision(small, precision):
    # FP32 inner heavy-ball solves inside the FP64 refinement, fixed m and adaptive
    for kw in (dict(m_init=512, adaptive=False), dict(m_init=8)):
        x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], method="polyak",
                            precision=precision, seed=1, max_iter=500, **kw)
        assert info["status"] == "ok", (kw, info)
        assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10


@pytest.mark.parametrize("precision", ["mixed", "mixed_fp32"])
def test_sjlt_mixed_precision(small, precision):
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], precision=precision, sketch="sjlt",
                        m_init=8, seed=1)
    assert info["status"] == "ok", info
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10


def test_cg_baseline(small):
    # the first steps follow the oracle's CG recurrence
    kw = dict(method="cg", stop="fixed", max_iter=10, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["iterations"] == io.iterations == 10 and info["final_m"] == 0 and info["resketches"] == 0
    assert reference.rel_error(x.cpu().numpy(), xo) <= 1e-10
    # to the stop rule: the error bound holds; the step count follows the oracle's closely (CG's
    # recurrences drift apart in the last bits over ~200 steps)
    kw = dict(method="cg", tol=1e-10, max_iter=5000)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], **kw)
    xo, io = solvers.solve(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok" and io.status == "ok"
    assert abs(info["iterations"] - io.iterations) <= max(5, io.iterations // 10)
    assert info["a_passes"] == info["iterations"]
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    # several right-hand sides (one recurrence per column)
    rng = np.random.default_rng(6)
    Bm = small["A"].T @ rng.standard_normal((4096, 3))
    X, info = aes.solve(small["dA"], to_dev(Bm), small["nu"], small["dlam"], **kw)
    Xr = reference.reference_solution(small["A"], Bm, small["nu"], small["lam"])
    assert info["status"] == "ok" and np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], method="cg", precision="mixed")
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], method="cg", stop="remark")


def test_wide_problem_two_product_path():
    # d > 8192: the steps use the two-product MFMA H.v (and no speculative enqueueing)
    P = synth.make_problem(12000, 8300, "geo:0.995", 1e-2, seed=17, backend="torch", device="cuda")
    Pn = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in P.items()}
    xr = reference.reference_solution(Pn["A"], Pn["b"], Pn["nu"], None, spectral=(Pn["V"], Pn["sigma"]))
    for method, sketch in (("pcg", "srht"), ("cg", "srht"), ("pcg", "srht_reuse"), ("polyak", "srht")):
        x, info = aes.solve(P["A"], P["b"], P["nu"], None, method=method, sketch=sketch, m_init=64, seed=3,
                            tol=1e-10, max_iter=3000)
        assert info["status"] == "ok", (method, sketch, info)
        assert reference.rel_error(x.cpu().numpy(), xr) <= 1e-10
        assert info["a_passes"] >= info["iterations"]


def test_lambda_and_ragged_shape():
    P = synth.make_problem(3000, 77, "pow:1", 1e-3, lam="uniform1_10", seed=5)
    xr = reference.reference_solution(P["A"], P["b"], P["nu"], P["lam"])
    kw = dict(m_init=2, seed=9, tol=1e-10)
    x, info = aes.solve(to_dev(P["A"]), to_dev(P["b"]), P["nu"], to_dev(P["lam"]), trace_cap=256, **kw)
    xo, io = solvers.adaptive_pcg(P["A"], P["b"], P["nu"], P["lam"], solvers.Options(**kw))
    assert _traj_gpu(info) == _traj_cpu(io)
    assert reference.rel_error(x.cpu().numpy(), xr) <= 1e-10


def test_multiple_rhs(small):
    rng = np.random.default_rng(4)
    Bm = small["A"].T @ rng.standard_normal((4096, 3))
    kw = dict(m_init=8, seed=4, tol=1e-10)
    X, info = aes.solve(small["dA"], to_dev(Bm), small["nu"], small["dlam"], trace_cap=256, **kw)
    Xo, io = solvers.adaptive_pcg(small["A"], Bm, small["nu"], small["lam"], solvers.Options(**kw))
    Xr = reference.reference_solution(small["A"], Bm, small["nu"], small["lam"])
    assert _traj_gpu(info) == _traj_cpu(io)
    assert np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)


@pytest.mark.parametrize("method", ["pcg", "ihs"])
def test_many_rhs_wide_vector_kernels(small, method):
    # 32 right-hand sides at d = 256: d * C = 8192, the grid form of the vector kernels
    rng = np.random.default_rng(11)
    Bm = small["A"].T @ rng.standard_normal((4096, 32))
    kw = dict(method=method, m_init=8, seed=6, tol=1e-10)
    X, info = aes.solve(small["dA"], to_dev(Bm), small["nu"], small["dlam"], trace_cap=256, **kw)
    Xo, io = solvers.solve(small["A"], Bm, small["nu"], small["lam"], solvers.Options(**kw))
    Xr = reference.reference_solution(small["A"], Bm, small["nu"], small["lam"])
    assert info["status"] == "ok"
    assert _traj_gpu(info) == _traj_cpu(io)
    assert np.all(reference.rel_error(X.cpu().numpy(), Xr) <= 1e-10)
    assert np.all(reference.rel_error(X.cpu().numpy(), Xo) <= 1e-9)


def test_forced_rejection_and_max_iter(small):
    kw = dict(m_init=512, seed=2, tol=1e-10, force_reject_at=3)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], trace_cap=256, **kw)
    xo, io = solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"],
                                  solvers.Options(m_init=512, seed=2, tol=1e-10, force_reject_at=(3,)))
    assert _traj_gpu(info) == _traj_cpu(io)
    assert info["a_passes"] == io.a_passes
    x3, info3 = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], m_init=8, seed=1, max_iter=3)
    xo3, io3 = solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"],
                                    solvers.Options(m_init=8, seed=1, max_iter=3))
    assert info3["status"] == "max_iter" and io3.status == "max_iter"
    assert reference.rel_error(x3.cpu().numpy(), xo3) <= 1e-8


def test_initialisation_stop_and_error_paths(small):
    """Paths where the step enqueued behind an initialisation must not run."""
    # zero right-hand side: the initialisation stops the only column, no step is taken
    zb = torch.zeros_like(small["db"])
    x, info = aes.solve(small["dA"], zb, small["nu"], small["dlam"], m_init=8, seed=1, trace_cap=8)
    xo, io = solvers.adaptive_pcg(small["A"], np.zeros_like(small["b"]), small["nu"], small["lam"],
                                  solvers.Options(m_init=8, seed=1))
    assert info["status"] == "ok" and info["attempts"] == 0 and info["trace"] == []
    assert info["a_passes"] == io.a_passes and float(x.abs().max()) == 0.0
    # no step allowed
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], m_init=8, seed=1, max_iter=0)
    assert info["status"] == "max_iter" and info["attempts"] == 0
    # a zero column and nu^2 below the smallest double: the Cholesky branch (m >= d) meets a
    # zero pivot, reported through the solver
    A = small["A"].copy()
    A[:, 0] = 0.0
    with pytest.raises(aes.AesError, match="not_spd"):
        aes.solve(to_dev(A), small["db"], 1e-200, None, m_init=512, seed=1)
    # the handle stays usable afterwards and reproduces the plain solve
    x1, info1 = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], m_init=8, seed=1)
    assert info1["status"] == "ok"
    assert reference.rel_error(x1.cpu().numpy(), small["xref"]) <= 1e-10


@pytest.mark.parametrize("stop", ["dtilde_rel", "fixed", "remark"])
def test_stop_rules(small, stop):
    tol = {"dtilde_rel": 1e-9, "fixed": 1e-10, "remark": 1e-12}[stop]
    kw = dict(m_init=8, seed=1, stop=stop, tol=tol, max_iter=12 if stop == "fixed" else 200)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], **kw)
    xo, io = solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(**kw))
    assert info["status"] == "ok" and io.status == "ok"
    assert info["iterations"] == io.iterations


def test_edge_cases(small):
    d = small["A"].shape[1]
    x, info = aes.solve(small["dA"], torch.zeros(d, dtype=torch.float64, device="cuda"), small["nu"])
    assert info["iterations"] == 0 and not torch.any(x)
    A1 = to_dev(np.array([[2.0]]))
    x, info = aes.solve(A1, to_dev(np.array([3.0])), 0.5)
    assert abs(x.item() - 3.0 / 4.25) < 1e-14
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], 0.0)
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], 1e-2, rho=1.0)
    with pytest.raises(aes.AesError, match="invalid_arg"):
        aes.solve(small["dA"], small["db"], 1e-2, -small["dlam"])


def test_x0_warm_start(small):
    x0 = small["xref"] + 1e-3 * np.random.default_rng(0).standard_normal(small["xref"].shape)
    kw = dict(m_init=8, seed=6, tol=1e-10)
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], x0=to_dev(x0), trace_cap=256, **kw)
    xo, io = solvers.adaptive_pcg(small["A"], small["b"], small["nu"], small["lam"], solvers.Options(x0=x0, **kw))
    assert _traj_gpu(info) == _traj_cpu(io)
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10


def test_deterministic(small):
    x1, _ = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], m_init=8, seed=1)
    x2, _ = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], m_init=8, seed=1)
    assert torch.equal(x1, x2)


def test_mixed_precision(small):
    x, info = aes.solve(small["dA"], small["db"], small["nu"], small["dlam"], precision="mixed", m_init=8, seed=1)
    assert info["status"] == "ok", info
    assert reference.rel_error(x.cpu().numpy(), small["xref"]) <= 1e-10
    assert info["refine_sweeps"] >= 2


@pytest.mark.parametrize("sketch", ["srht", "srht_nested"])
def test_batched_equals_singles(sketch):
    probs = []
    for i, (n, d) in enumerate([(2048, 64), (3000, 128), (1024, 256)]):
        P = synth.make_problem(n, d, "geo:0.98", 10.0 ** (-1 - i), nrhs=2, seed=20 + i)
        probs.append(dict(A=to_dev(P["A"]), b=to_dev(P["b"]), nu=P["nu"], xref=reference.reference_solution(
            P["A"], P["b"], P["nu"])))
    res = aes.solve_batched(probs, tol=1e-10, m_init=16, seed=3, sketch=sketch)
    for p, (x, info) in enumerate(res):
        assert info["status"] == "ok"
        assert np.all(reference.rel_error(x.cpu().numpy(), probs[p]["xref"]) <= 1e-10)
        xs, _ = aes.solve(probs[p]["A"], probs[p]["b"], probs[p]["nu"], m_init=16, seed=3, problem=p, sketch=sketch)
        assert torch.equal(xs, x)


# the adjoint solve runs the forward solve's method and sketch
@pytest.mark.parametrize("opts", [dict(m_init=16), dict(m_init=16, sketch="srht_reuse"),
                                  dict(m_init=16, sketch="srht_nested"),
                                  dict(method="polyak", m_init=512, adaptive=False)])
def test_autograd_adjoint(opts):
    P = synth.make_problem(2048, 64, "pow:0.5", 1e-2, seed=31, with_xt=True)
    A, b, nu, xt = P["A"], P["b"], P["nu"], P["xt"]
    At = to_dev(A).requires_grad_(True)
    bt = to_dev(b).requires_grad_(True)
    ln = torch.tensor(np.log(nu), dtype=torch.float64, device="cuda", requires_grad=True)
    x = aes.SketchSolve.apply(At, bt, ln, None, dict(seed=2, tol=1e-12, **opts))
    loss = 0.5 * torch.sum((x - to_dev(xt)) ** 2)
    loss.backward()
    xs = reference.reference_solution(A, b, nu)
    _, adj, db, dA, dln = adjoint.gradients(A, b, nu, xs - xt, x=xs)
    assert np.max(np.abs(bt.grad.cpu().numpy() - db)) <= 1e-9 * np.max(np.abs(db))
    assert np.max(np.abs(At.grad.cpu().numpy() - dA)) <= 1e-9 * np.max(np.abs(dA))
    assert abs(ln.grad.item() - dln) <= 1e-9 * abs(dln)
