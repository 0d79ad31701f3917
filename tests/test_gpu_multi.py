"""Multi-RHS products, FP32-storage mixed precision and the concurrent batched driver."""
import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
import synth
from oracle import reference

from _helpers import to_dev

pytestmark = pytest.mark.gpu
U32 = np.finfo(np.float32).eps / 2


@pytest.mark.parametrize("n,d,c", [(1000, 64, 2), (5000, 300, 4), (9000, 256, 32), (70, 129, 8)])
def test_hv_multi_fp64(n, d, c):
    rng = np.random.default_rng(n + c)
    A = rng.standard_normal((n, d))
    P = rng.standard_normal((d, c))
    lam = 1 + rng.random(d)
    Q = aes.hv_multi(to_dev(A), to_dev(P), 0.2, to_dev(lam)).cpu().numpy()
    ref = A.T @ (A @ P) + 0.04 * lam[:, None] * P
    mag = np.abs(A).T @ (np.abs(A) @ np.abs(P)) + 0.04 * lam[:, None] * np.abs(P)
    k = n + d + 8
    assert np.all(np.abs(Q - ref) <= 2 * k * 1.12e-16 * mag)


@pytest.mark.parametrize("n,d,c", [(1000, 64, 1), (5000, 300, 4), (9000, 256, 32), (70, 129, 8)])
def test_hv_multi_fp32_storage(n, d, c):
    # reference: the exact product with A and P rounded to FP32 (what the FP32 path multiplies)
    rng = np.random.default_rng(n + 3 * c)
    A = rng.standard_normal((n, d))
    P = rng.standard_normal((d, c))
    A32 = A.astype(np.float32).astype(np.float64)
    P32 = P.astype(np.float32).astype(np.float64)
    Q = aes.hv_multi(to_dev(A), to_dev(P), 0.2, None, precision="mixed_fp32").cpu().numpy()
    ref = A32.T @ (A32 @ P32) + 0.04 * P
    mag = np.abs(A32).T @ (np.abs(A32) @ np.abs(P32)) + 0.04 * np.abs(P)
    k = d + 4096 + 8  # FP32 accumulation over a row of A and over one row block
    assert np.all(np.abs(Q - ref) <= 2 * k * U32 * mag)


@pytest.mark.parametrize("precision,c", [("mixed_fp32", 4), ("mixed", 2), ("mixed_fp32", 1)])
def test_mixed_multi_rhs(precision, c):
    P = synth.make_problem(4096, 256, "geo:0.98", 1e-3, nrhs=c, seed=50)
    xr = reference.reference_solution(P["A"], P["b"], P["nu"])
    x, info = aes.solve(to_dev(P["A"]), to_dev(P["b"]), P["nu"], precision=precision, m_init=16, seed=2)
    assert info["status"] == "ok", info
    assert np.all(reference.rel_error(x.cpu().numpy(), xr) <= 1e-10)


def test_batched_mixed_fp32_uneven():
    specs = [(4096, 256, 1e-1), (6144, 512, 1e-4), (2048, 256, 1e-3), (8192, 768, 1e-2), (3072, 512, 3e-3)]
    probs = []
    for i, (n, d, nu) in enumerate(specs):
        P = synth.make_problem(n, d, "geo:0.98", nu, nrhs=32, seed=60 + i)
        probs.append(dict(A=to_dev(P["A"]), b=to_dev(P["b"]), nu=nu, A_np=P["A"], b_np=P["b"], V=P["V"],
                          sigma=P["sigma"]))
    res = aes.solve_batched(probs, tol=1e-10, precision="mixed_fp32", m_init=16, seed=5)
    for p, (x, info) in enumerate(res):
        assert info["status"] == "ok", (p, info)
        xr = reference.reference_solution(probs[p]["A_np"], probs[p]["b_np"], probs[p]["nu"],
                                          spectral=(probs[p]["V"], probs[p]["sigma"]))
        err = reference.rel_error(x.cpu().numpy(), xr)
        assert np.all(err <= 1e-10), (p, float(err.max()))
    # concurrency does not change any result: equal to the single solve of problem p
    for p in (0, 3):
        xs, _ = aes.solve(probs[p]["A"], probs[p]["b"], probs[p]["nu"], precision="mixed_fp32", m_init=16, seed=5,
                          problem=p)
        assert torch.equal(xs, res[p][0])
