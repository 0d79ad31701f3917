"""Argument checks and resource ownership of the torch-facing wrappers (GPU)."""
import gc
import threading

import pytest
import torch

import paper_2104_14101_amd as aes
import synth

pytestmark = pytest.mark.gpu


def _problem(n=2048, d=128, seed=7):
    P = synth.make_problem(n, d, "geo:0.9", 1e-2, seed=seed)
    return torch.from_numpy(P["A"]).cuda(), torch.from_numpy(P["b"]).cuda(), P["nu"]


@pytest.mark.parametrize("bad", ["cpu", "f32", "short"])
def test_lambda_checked_in_every_entry_point(bad):
    A, b, nu = _problem()
    d = A.shape[1]
    lam = {"cpu": torch.ones(d, dtype=torch.float64), "f32": torch.ones(d, dtype=torch.float32, device="cuda"),
           "short": torch.ones(d - 1, dtype=torch.float64, device="cuda")}[bad]
    exc = ValueError if bad == "short" else TypeError
    SA = aes.sketch(A, 256, seed=1)
    P = torch.randn(d, 4, dtype=torch.float64, device="cuda")
    calls = [
        lambda: aes.solve(A, b, nu, lam),
        lambda: aes.solve_dual(A[:64].contiguous(), b, nu, lam),
        lambda: aes.solve_batched([dict(A=A, b=b, nu=nu, lam=lam)]),
        lambda: aes.hv(A, b, nu, lam),
        lambda: aes.hv_multi(A, P, nu, lam),
        lambda: aes.factor(SA, nu, lam),
        lambda: aes.precond_apply(SA, nu, lam, b),
        lambda: aes.SketchSolve.apply(A, b.clone().requires_grad_(True), torch.tensor(0.0, dtype=torch.float64,
                                                                                     device="cuda"), lam, {}),
    ]
    for f in calls:
        with pytest.raises(exc):
            f()


def test_out_buffer_checked():
    A, b, nu = _problem()
    d = A.shape[1]
    for x in [torch.empty(d, dtype=torch.float32, device="cuda"), torch.empty(d, dtype=torch.float64),
              torch.empty(d + 1, dtype=torch.float64, device="cuda"),
              torch.empty(2 * d, dtype=torch.float64, device="cuda")[::2]]:
        with pytest.raises((TypeError, ValueError)):
            aes.solve(A, b, nu, x=x)
    x = torch.empty(d, dtype=torch.float64, device="cuda")
    out, info = aes.solve(A, b, nu, x=x, m_init=8, seed=3)
    assert out is x and info["status"] == "ok"


def test_no_grad_forwards_hold_no_device_memory():
    A, b, nu = _problem(4096, 256, 3)
    ln = torch.log(torch.tensor(nu, dtype=torch.float64, device="cuda"))
    Ar = A.clone().requires_grad_(True)
    # warm both routes: the shared handle's pool (no-grad solve) and a kept context (dropped)
    with torch.no_grad():
        x0 = aes.SketchSolve.apply(Ar, b, ln, None, dict(m_init=8, seed=1))
    x0 = aes.SketchSolve.apply(Ar, b, ln, None, dict(m_init=8, seed=1))
    del x0
    gc.collect()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with torch.no_grad():
        for _ in range(4):
            x = aes.SketchSolve.apply(Ar, b, ln, None, dict(m_init=8, seed=1))
    del x
    for _ in range(4):  # outputs dropped without a backward: the kept contexts are released
        y = aes.SketchSolve.apply(Ar, b, ln, None, dict(m_init=8, seed=1))
        del y
    gc.collect()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0


def test_second_backward_with_retained_graph():
    A, b, nu = _problem(4096, 256, 5)
    Ar = A.clone().requires_grad_(True)
    br = b.clone().requires_grad_(True)
    ln = torch.log(torch.tensor(nu, dtype=torch.float64, device="cuda")).requires_grad_(True)
    x = aes.SketchSolve.apply(Ar, br, ln, None, dict(m_init=8, seed=2, tol=1e-12))
    loss = 0.5 * (x * x).sum()
    g1 = torch.autograd.grad(loss, (Ar, br, ln), retain_graph=True)
    g2 = torch.autograd.grad(loss, (Ar, br, ln))
    for a, c in zip(g1, g2):
        assert torch.allclose(a, c, rtol=1e-9, atol=0)


def test_threads_share_the_handle():
    A, b, nu = _problem(4096, 256, 9)
    ref, _ = aes.solve(A, b, nu, m_init=8, seed=4)
    torch.cuda.synchronize()
    out = [None] * 4

    def run(i):
        x, _ = aes.solve(A, b, nu, m_init=8, seed=4)
        torch.cuda.synchronize()
        out[i] = x

    th = [threading.Thread(target=run, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for x in out:
        assert torch.equal(x, ref)


def test_keep_fp32_copy_reuses_only_the_same_matrix():
    A, b, nu = _problem(8192, 256, 11)
    opts = dict(precision="mixed", m_init=8, seed=2)
    x_ref, i_ref = aes.solve(A, b, nu, **opts)
    x1, i1 = aes.solve(A, b, nu, keep_fp32_copy=True, **opts)  # the copy cast by the first solve
    assert i_ref["status"] == "ok" and i1["status"] == "ok"
    assert torch.equal(x1, x_ref)
    # another matrix of the same shape at another address: cast again despite the option
    A2 = A * 0.5
    x2, _ = aes.solve(A2, b, nu, keep_fp32_copy=True, **opts)
    x2_ref, _ = aes.solve(A2.clone(), b, nu, **opts)
    assert torch.equal(x2, x2_ref)
    # without the promise an in-place change is always seen
    A.mul_(0.5)
    x3, _ = aes.solve(A, b, nu, **opts)
    assert torch.equal(x3, x2_ref)
