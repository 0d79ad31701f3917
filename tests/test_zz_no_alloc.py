"""aes_hv_noalloc (the allocation-free fused H.v) against aes_hv, through the C ABI.

Both run the same kernels in the same grid, so their outputs must be bit-identical; two calls
in a row with the second on a smaller input (the static workspace keeps the first call's
partials), plus the oracle's product as a sanity check and the argument errors.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
from paper_2104_14101_amd import _binding as B

from _helpers import hv_bound, to_dev

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _call(name, A, p, nu, lam, q, php):
    lib = B.load()
    dev = A.device
    h = aes._handle(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    n, d = A.shape
    st = getattr(lib, name)(h, stream, n, d, _vp(A), A.stride(0), float(nu), _vp(lam), _vp(p), _vp(q), _vp(php))
    return st


def _case(n, d, seed, with_lam):
    g = torch.Generator("cuda").manual_seed(seed)
    A = torch.randn(n, d, dtype=torch.float64, device="cuda", generator=g)
    p = torch.randn(d, dtype=torch.float64, device="cuda", generator=g)
    lam = (1 + 9 * torch.rand(d, dtype=torch.float64, device="cuda", generator=g)) if with_lam else None
    return A, p, lam


def _both(A, p, nu, lam):
    d = A.shape[1]
    q0 = torch.full((d,), float("nan"), dtype=torch.float64, device="cuda")
    p0 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    q1 = torch.full((d,), float("nan"), dtype=torch.float64, device="cuda")
    p1 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    assert _call("aes_hv_noalloc", A, p, nu, lam, q1, p1) == B.AES_OK
    assert _call("aes_hv", A, p, nu, lam, q0, p0) == B.AES_OK
    torch.cuda.synchronize()
    return q0, p0, q1, p1


def test_noalloc_matches_aes_hv_two_calls():
    # first call: the bench shape with Lambda; second: smaller, ragged, Lambda = I
    for n, d, seed, with_lam, nu in [(65536, 2048, 1, True, 1e-3), (3001, 701, 2, False, 0.37)]:
        A, p, lam = _case(n, d, seed, with_lam)
        q0, p0, q1, p1 = _both(A, p, nu, lam)
        assert torch.equal(q0, q1), (n, d)
        assert torch.equal(p0, p1), (n, d)
        if n <= 4096:
            An, pn = A.cpu().numpy(), p.cpu().numpy()
            ln = lam.cpu().numpy() if lam is not None else None
            qref = An.T @ (An @ pn) + nu ** 2 * (ln if ln is not None else 1.0) * pn
            assert np.all(np.abs(q1.cpu().numpy() - qref) <= hv_bound(An, ln, nu, pn))


def test_noalloc_widest_and_no_pHp():
    A, p, lam = _case(777, 8192, 3, True)
    q0, p0, q1, p1 = _both(A, p, 0.5, lam)
    assert torch.equal(q0, q1) and torch.equal(p0, p1)
    q2 = torch.empty_like(q1)
    assert _call("aes_hv_noalloc", A, p, 0.5, lam, q2, None) == B.AES_OK
    torch.cuda.synchronize()
    assert torch.equal(q2, q1)


def test_noalloc_allocates_nothing():
    A, p, lam = _case(20000, 1024, 4, True)
    q = torch.empty(1024, dtype=torch.float64, device="cuda")
    php = torch.empty(1, dtype=torch.float64, device="cuda")
    assert _call("aes_hv_noalloc", A, p, 0.1, lam, q, php) == B.AES_OK  # kernels loaded
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        assert _call("aes_hv_noalloc", A, p, 0.1, lam, q, php) == B.AES_OK
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_noalloc_rejects_wide_d():
    A, p, lam = _case(16, 8193, 5, False)
    q = torch.full((8193,), 7.0, dtype=torch.float64, device="cuda")
    assert _call("aes_hv_noalloc", A, p, 0.1, None, q, None) == B.AES_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((q == 7.0).all())
