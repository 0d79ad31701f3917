"""Full-size workloads: the solution (or gradient) against the oracle's refined reference.

Inputs are drawn on the GPU (the QR factorisations of the generator would dominate a CPU
run); the oracle runs on the host copies.  Each test prints the case it runs."""
import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
import synth

from _helpers import spectral_error
from oracle import adjoint, reference

pytestmark = pytest.mark.gpu


def _np(P):
    return {k: (v.detach().cpu().numpy() if hasattr(v, "detach") else v) for k, v in P.items()}


@pytest.fixture(scope="module")
def pcg_workload():
    P = synth.make_workload("pcg_n65536_d2048", seed=0, backend="torch", device="cuda")
    Pn = _np(P)
    Pn["xref"] = reference.reference_solution(Pn["A"], Pn["b"], Pn["nu"], Pn["lam"])
    return P, Pn


@pytest.mark.parametrize("method,kind", [("pcg", "srht"), ("ihs", "srht"), ("pcg", "gauss"), ("ihs", "gauss")])
def test_n65536_d2048(pcg_workload, method, kind):
    P, Pn = pcg_workload
    print(f"case n=65536 d=2048 {method} {kind}", flush=True)
    x, info = aes.solve(P["A"], P["b"], P["nu"], P["lam"], method=method, sketch=kind, m_init=16, seed=1)
    err = float(reference.rel_error(x.cpu().numpy(), Pn["xref"]))
    print(f"  status={info['status']} t={info['iterations']} m={info['final_m']} err={err:.2e}", flush=True)
    assert info["status"] == "ok" and err <= 1e-10


def test_n262144_d4096_fp64_and_mixed():
    print("case n=262144 d=4096 fp64 + mixed", flush=True)
    P = synth.make_workload("mixed_n262144_d4096", seed=0, backend="torch", device="cuda")
    Pn = _np(P)
    xr = reference.reference_solution(Pn["A"], Pn["b"], Pn["nu"], None, spectral=(Pn["V"], Pn["sigma"]))
    for prec in ("fp64", "mixed"):
        x, info = aes.solve(P["A"], P["b"], P["nu"], precision=prec, m_init=16, seed=1)
        err = float(reference.rel_error(x.cpu().numpy(), xr))
        print(f"  {prec}: status={info['status']} m={info['final_m']} sweeps={info['refine_sweeps']} err={err:.2e}",
              flush=True)
        assert info["status"] == "ok" and err <= 1e-10


@pytest.mark.timeout(1500)
def test_batched_all_64_problems_32_rhs():
    # every (problem, right-hand side) pair of the batched workload within 1e-10 of x*: the
    # oracle's extended-precision residual of the GPU result, mapped through the exact spectral
    # inverse of each problem
    specs = synth.batched_specs(64, seed=0)
    probs = []
    for i, sp in enumerate(specs):
        P = synth.make_problem(sp["n"], sp["d"], sp["decay"], sp["nu"], nrhs=32, seed=1000 + i, backend="torch",
                               device="cuda")
        probs.append(P)
    print("case batched 64 x 32 rhs, mixed_fp32", flush=True)
    res = aes.solve_batched([dict(A=P["A"], b=P["b"], nu=P["nu"]) for P in probs], tol=1e-10,
                            precision="mixed_fp32", m_init=16, seed=7)
    worst = 0.0
    for i, (P, (x, info)) in enumerate(zip(probs, res)):
        assert info["status"] == "ok", (i, info)
        err = spectral_error(P["A"].cpu().numpy(), P["b"].cpu().numpy(), P["nu"], P["V"].cpu().numpy(), P["sigma"],
                             x.cpu().numpy(), threads=16)
        worst = max(worst, float(err.max()))
        print(f"  problem {i} n={specs[i]['n']} d={specs[i]['d']} nu={specs[i]['nu']:.1e} m={info['final_m']} "
              f"sweeps={info['refine_sweeps']} max err over 32 rhs={err.max():.2e}", flush=True)
        assert np.all(err <= 1e-10), (i, float(err.max()))
        probs[i] = None  # free the problem's device memory as the check goes
    print(f"  weakest pair: {worst:.2e}", flush=True)


def test_adjoint_n131072_d1024():
    print("case autograd n=131072 d=1024", flush=True)
    P = synth.make_workload("adjoint_n131072_d1024", seed=0, backend="torch", device="cuda", with_xt=True)
    A = P["A"].clone().requires_grad_(True)
    b = P["b"].clone().requires_grad_(True)
    ln = torch.tensor(np.log(P["nu"]), dtype=torch.float64, device="cuda", requires_grad=True)
    x = aes.SketchSolve.apply(A, b, ln, None, dict(m_init=16, seed=3, tol=1e-12))
    loss = 0.5 * torch.sum((x - P["xt"]) ** 2)
    loss.backward()
    Pn = _np(P)
    xs = reference.reference_solution(Pn["A"], Pn["b"], Pn["nu"], None, spectral=(Pn["V"], Pn["sigma"]))
    _, adj, db, dA, dln = adjoint.gradients(Pn["A"], Pn["b"], Pn["nu"], xs - Pn["xt"], x=xs)
    eb = np.max(np.abs(b.grad.cpu().numpy() - db)) / np.max(np.abs(db))
    eA = np.max(np.abs(A.grad.cpu().numpy() - dA)) / np.max(np.abs(dA))
    eln = abs(ln.grad.item() - dln) / abs(dln)
    print(f"  rel errors: db={eb:.2e} dA={eA:.2e} dlognu={eln:.2e}", flush=True)
    assert eb <= 1e-9 and eA <= 1e-9 and eln <= 1e-9
