"""Kernel-level parity of the HIP library against the oracle (called through the C ABI)."""
import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
import synth
from oracle import factor as ofac
from oracle import philox
from oracle import sketch as osk

from _helpers import U, hv_bound, to_dev

pytestmark = pytest.mark.gpu


# d > 8192: the two-pass form (odd d: scalar loads; 9000: ragged last column block)
@pytest.mark.parametrize("n,d", [(1, 1), (37, 5), (1000, 256), (777, 300), (3001, 1024), (1500, 2048), (513, 4096),
                                 (64, 4097), (700, 9000), (333, 8193)])
def test_hv_matches_oracle(n, d):
    rng = np.random.default_rng(n * 7 + d)
    A = rng.standard_normal((n, d))
    p = rng.standard_normal(d)
    lam = 1 + 9 * rng.random(d)
    nu = 0.37
    q, php = aes.hv(to_dev(A), to_dev(p), nu, to_dev(lam))
    torch.cuda.synchronize()
    qref = A.T @ (A @ p) + nu ** 2 * lam * p
    bound = hv_bound(A, lam, nu, p)
    assert np.all(np.abs(q.cpu().numpy() - qref) <= bound)
    Ap = A @ p
    pref = Ap @ Ap + nu ** 2 * p @ (lam * p)
    assert abs(php.item() - pref) <= 4 * (n + d) * 1.2e-16 * pref


def test_hv_strided_rows():
    rng = np.random.default_rng(3)
    big = rng.standard_normal((500, 300))
    A = to_dev(big)[:, :257]  # lda = 300, odd d
    p = rng.standard_normal(257)
    q, _ = aes.hv(A, to_dev(p), 0.1)
    qref = big[:, :257].T @ (big[:, :257] @ p) + 0.01 * p
    assert np.all(np.abs(q.cpu().numpy() - qref) <= hv_bound(big[:, :257], None, 0.1, p))


def test_hv_full_size_pcg_workload():
    P = synth.make_problem(65536, 2048, "pow:1", 1e-3, lam="uniform1_10", seed=11, backend="torch", device="cuda")
    A = P["A"]
    p = torch.randn(2048, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    q, _ = aes.hv(A, p, 1e-3, P["lam"])
    An, pn, ln = A.cpu().numpy(), p.cpu().numpy(), P["lam"].cpu().numpy()
    qref = An.T @ (An @ pn) + 1e-6 * ln * pn
    assert np.all(np.abs(q.cpu().numpy() - qref) <= hv_bound(An, ln, 1e-3, pn))


@pytest.mark.parametrize("n,d,m", [(1, 3, 1), (8, 4, 4), (1000, 40, 16), (513, 33, 64), (5000, 17, 256),
                                   (70000, 8, 1024), (300000, 3, 64)])
def test_srht_bit_exact_on_integers(n, d, m):
    # Integer data: every FWHT partial sum is exact in FP64; sqrt(m) is a power of two.
    rng = np.random.default_rng(n + d + m)
    A = rng.integers(-50, 51, size=(n, d)).astype(np.float64)
    SA = aes.sketch(to_dev(A), m, "srht", seed=99, k=3).cpu().numpy()
    ref = osk.srht(A, m, 99, 3)
    np.testing.assert_array_equal(SA, ref)


@pytest.mark.parametrize("n,d,m", [(4096, 256, 1024), (3000, 70, 100), (20000, 129, 1000)])
def test_srht_float_data(n, d, m):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, d))
    SA = aes.sketch(to_dev(A), m, "srht", seed=4, k=1).cpu().numpy()
    ref = osk.srht(A, m, 4, 1)
    # Both sides apply the radix-2 stages in the same bit order, so the transform is
    # bit-identical; only the final 1/sqrt(m) (a multiply vs a divide) may round differently.
    np.testing.assert_allclose(SA, ref, rtol=4.5e-16, atol=0)


@pytest.mark.parametrize("n,d,m,k", [(4000, 33, 1024, 3), (16384, 64, 256, 0), (16384, 64, 256, 5)])
def test_srht_reuse_bit_exact_on_integers(n, d, m, k):
    # n' and n'/m powers of 4: the normalised transform and the rescale by sqrt(n'/m) are exact
    rng = np.random.default_rng(n + d + m + k)
    A = rng.integers(-50, 51, size=(n, d)).astype(np.float64)
    SA = aes.sketch(to_dev(A), m, "srht_reuse", seed=21, k=k).cpu().numpy()
    np.testing.assert_array_equal(SA, osk.srht_reuse(A, m, 21, k))


@pytest.mark.parametrize("n,d,m,k", [(3000, 70, 100, 2), (20000, 129, 1000, 1)])
def test_srht_reuse_float_data(n, d, m, k):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((n, d))
    SA = aes.sketch(to_dev(A), m, "srht_reuse", seed=4, k=k).cpu().numpy()
    # identical transform; the two scalings may each round differently
    np.testing.assert_allclose(SA, osk.srht_reuse(A, m, 4, k), rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,d,m", [(4000, 33, 1024), (16384, 64, 256), (16384, 64, 16384), (13, 3, 4), (3, 2, 1)])
def test_srht_nested_bit_exact_on_integers(n, d, m):
    # n' and n'/m powers of 4: exact transform and rescale; the row order (the device's bucket
    # sort of the row keys) must equal the oracle's stable argsort, prefix by prefix
    rng = np.random.default_rng(n + d + m + 1)
    A = rng.integers(-50, 51, size=(n, d)).astype(np.float64)
    for k in (0, 3):  # the sketch index plays no part
        SA = aes.sketch(to_dev(A), m, "srht_nested", seed=21, k=k).cpu().numpy()
        np.testing.assert_array_equal(SA, osk.srht_nested(A, m, 21))


@pytest.mark.parametrize("n,d,m", [(3000, 70, 100), ((1 << 20) + 5, 4, 1 << 20)])
def test_srht_nested_float_data(n, d, m):
    # the second case has n' = 2^21: 2048 blocks of the bucket-count scan (two chunks of the
    # block-total scan) and a million rows whose order is checked
    rng = np.random.default_rng(7)
    A = rng.standard_normal((n, d))
    SA = aes.sketch(to_dev(A), m, "srht_nested", seed=4, k=0).cpu().numpy()
    np.testing.assert_allclose(SA, osk.srht_nested(A, m, 4), rtol=1e-15, atol=0)


def test_srht_full_size_sampled_rows():
    P = synth.make_problem(65536, 2048, "pow:1", 1e-3, seed=12, backend="torch", device="cuda")
    A = P["A"]
    m = 4096
    SA = aes.sketch(A, m, "srht", seed=5, k=2).cpu().numpy()
    An = A.cpu().numpy()
    for j in (0, 1, 777, 4095):
        ref = osk.srht_row(An, m, 5, 2, j)
        assert np.max(np.abs(SA[j] - ref)) <= 1e-13 * np.max(np.abs(ref)) * 16


# (2000, 130, 512): 32 split-K ranges, the last one ragged
@pytest.mark.parametrize("n,d,m", [(300, 40, 70), (1000, 65, 128), (129, 7, 3), (2000, 130, 512)])
def test_gaussian_sketch(n, d, m):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((n, d))
    SA = aes.sketch(to_dev(A), m, "gauss", seed=8, k=2).cpu().numpy()
    ref = osk.gaussian(A, m, 8, 2)
    # G entries agree to a few ulps (device and host libm), sums of n terms
    assert np.max(np.abs(SA - ref)) <= 1e-13 * np.sqrt(n) * np.max(np.abs(ref)) + 1e-14


# (10000, 256, 8192): three generated slabs of four split-K ranges, the last slab ragged;
# (65536, 2048, 16383): the bench workload's largest sketch (32 slabs, one split, m ragged)
@pytest.mark.parametrize("n,d,m", [(10000, 256, 8192), (65536, 2048, 16383)])
def test_gaussian_sampled_rows(n, d, m):
    P = synth.make_problem(n, d, "pow:1", 1e-3, seed=13, backend="torch", device="cuda")
    A = P["A"]
    SA = aes.sketch(A, m, "gauss", seed=9, k=3).cpu().numpy()
    An = A.cpu().numpy()
    rows = np.array([0, 1, 5, m // 2 + 3, m - 1])
    ref = philox.gaussian_rows(9, 3, rows, 0, n) @ An / np.sqrt(m)
    assert np.max(np.abs(SA[rows] - ref)) <= 1e-13 * np.sqrt(n) * np.max(np.abs(ref)) + 1e-14


def _sjlt_bound(A, h, m):
    # |fl(sum) - sum| <= (k - 1) u sum |terms| for any order of k terms; k <= bucket size
    absum = np.zeros((m, A.shape[1]))
    np.add.at(absum, h, np.abs(A))
    cnt = np.bincount(h, minlength=m)[:, None]
    return cnt * 2.0 ** -53 * absum


# one piece per bucket (Q = 1: the sums run in the oracle's order, bit for bit) and several
# (Q > 1: pieces summed in order); odd d and lda (scalar loads), m > n (empty buckets), m = 1,
# several counting blocks with a ragged last one
@pytest.mark.parametrize("n,d,m,exact", [(300, 40, 70, True), (129, 7, 3, True), (3000, 257, 4096, True),
                                         (70000, 64, 4096, True), (1000, 65, 7, False), (5000, 130, 1, False),
                                         (70000, 33, 1024, False)])
def test_sjlt_sketch(n, d, m, exact):
    rng = np.random.default_rng(n + d + m)
    A = rng.standard_normal((n, d))
    SA = aes.sketch(to_dev(A), m, "sjlt", seed=8, k=2).cpu().numpy()
    ref = osk.sjlt(A, m, 8, 2)
    if exact:
        np.testing.assert_array_equal(SA, ref)
    else:
        h, _ = philox.sjlt_hash(8, 2, n, m)
        assert np.all(np.abs(SA - ref) <= _sjlt_bound(A, h, m))


@pytest.mark.parametrize("kind", ["sjlt", "gauss", "srht"])
def test_sketch_strided_rows(kind):
    # A as a column slice of a wider matrix: lda = 300 > d = 257 (odd: scalar loads)
    rng = np.random.default_rng(21)
    big = rng.standard_normal((1200, 300))
    A = to_dev(big)[:, :257]
    SA = aes.sketch(A, 100, kind, seed=4, k=1).cpu().numpy()
    ref = osk.sketch(big[:, :257], 100, kind, 4, 1)
    assert np.max(np.abs(SA - ref)) <= 1e-13 * np.sqrt(1200) * np.max(np.abs(ref))


@pytest.mark.parametrize("m", [16384, 16])
def test_sjlt_full_size_sampled_rows(m):
    P = synth.make_problem(65536, 2048, "pow:1", 1e-3, seed=14, backend="torch", device="cuda")
    A = P["A"]
    SA = aes.sketch(A, m, "sjlt", seed=5, k=4).cpu().numpy()
    An = A.cpu().numpy()
    h, sgn = philox.sjlt_hash(5, 4, 65536, m)
    for r in (0, 1, m // 2 + 1, m - 1):
        idx = np.nonzero(h == r)[0]
        acc = np.zeros(2048)
        for i in idx:  # increasing row order from zero, as the definition sums
            acc = acc + sgn[i] * An[i]
        if m * 64 >= 65536:
            np.testing.assert_array_equal(SA[r], acc)
        else:
            bound = len(idx) * 2.0 ** -53 * np.abs(An[idx]).sum(axis=0)
            assert np.all(np.abs(SA[r] - acc) <= bound)


@pytest.mark.parametrize("m,d", [(200, 100), (100, 100), (37, 100), (1, 5), (300, 257), (129, 130)])
def test_factor_and_apply(m, d):
    rng = np.random.default_rng(m + d)
    SA = rng.standard_normal((m, d)) / np.sqrt(m)
    lam = 1 + rng.random(d)
    nu = 0.05
    G, L = aes.factor(to_dev(SA), nu, to_dev(lam))
    P = ofac.SketchedHessian(SA, nu, lam)
    Lref = P.L
    Gn = G.cpu().numpy()
    if m >= d:
        Gref = SA.T @ SA + nu ** 2 * np.diag(lam)
    else:
        Gref = (SA / lam) @ SA.T + nu ** 2 * np.eye(m)
    np.testing.assert_allclose(np.tril(Gn), np.tril(Gref), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(L.cpu().numpy(), Lref, rtol=1e-9, atol=1e-11)
    for c in (1, 2, 4, 8):
        z = rng.standard_normal((d, c))
        v = aes.precond_apply(to_dev(SA), nu, to_dev(lam), to_dev(z)).cpu().numpy()
        vref = P.apply(z)
        np.testing.assert_allclose(v, vref, rtol=1e-8, atol=1e-10 * np.max(np.abs(vref)))


def test_factor_not_spd_is_reported():
    SA = np.zeros((4, 6))
    with pytest.raises(aes.AesError, match="not_spd"):
        aes.factor(to_dev(SA), 1e-200, None)  # nu^2 underflows to 0: a zero pivot


def test_philox_streams_on_device_match_oracle():
    # signs and row selection are checked through the SRHT of the identity (H E columns)
    n = 64
    I = np.eye(n)
    SA = aes.sketch(to_dev(I), 16, "srht", seed=2**63 + 5, k=7, problem=3).cpu().numpy()
    ref = osk.srht(I, 16, 2**63 + 5, 7, problem=3)
    np.testing.assert_array_equal(SA, ref)
    eps = philox.signs(2**63 + 5, 7, n, problem=3)
    assert np.all(np.sign(SA[0]) == np.sign(ref[0])) and set(np.unique(eps)) <= {-1.0, 1.0}


# (c = 1 with even d takes the single-pass form, the others the two-pass one)
@pytest.mark.parametrize("n,d,c,nu,with_lam", [(16384, 2048, 4, 1e-4, False), (3000, 257, 1, 1e-3, True),
                                               (777, 96, 32, 1e-2, True), (20000, 4096, 1, 1e-4, False),
                                               (5000, 1000, 1, 1e-3, True), (4100, 300, 8, 1e-3, False),
                                               (2050, 520, 16, 1e-2, True)])
def test_compensated_residual_matches_the_extended_oracle(n, d, c, nu, with_lam):
    # near the solution b - H x is a tiny difference of terms of the size of H x (kappa(H) ~ 1e8
    # for the first, batched-workload-like shape): the compensated FP64 residual agrees with the
    # oracle's 64-bit-significand one to within their rounding bounds, which plain FP64 misses
    from oracle import reference

    P = synth.make_problem(n, d, "geo:0.98", nu, nrhs=c, seed=31, lam="uniform1_10" if with_lam else "identity")
    A, b = P["A"], P["b"].reshape(d, c)
    lam = P["lam"] if with_lam else None
    xr = reference.reference_solution(A, b, nu, lam)
    x = xr * (1.0 + 1e-12 * np.random.default_rng(2).standard_normal(xr.shape))
    r_ref = reference.residual_extended(A, b, nu, lam, x)
    rd = torch.empty((d, c), dtype=torch.float64, device="cuda")
    from paper_2104_14101_amd import _binding as B
    import ctypes

    h = aes._handle(torch.device("cuda:0"))
    At, bt, xt = to_dev(A), to_dev(b), to_dev(x)
    lt = to_dev(lam) if with_lam else None
    st = B.load().aes_residual(h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), n, d, c,
                               ctypes.c_void_p(At.data_ptr()), d, ctypes.c_void_p(bt.data_ptr()), c, nu,
                               ctypes.c_void_p(lt.data_ptr() if lt is not None else 0),
                               ctypes.c_void_p(xt.data_ptr()), c, ctypes.c_void_p(rd.data_ptr()), c)
    assert st == B.AES_OK
    torch.cuda.synchronize()
    r_gpu = rd.cpu().numpy()
    lamv = np.ones(d) if lam is None else lam
    mag = np.abs(A).T @ (np.abs(A) @ np.abs(x)) + nu ** 2 * lamv[:, None] * np.abs(x) + np.abs(b)
    k = n + d + 8
    uld = 2.0 ** -64
    bound = 2 * U * np.abs(r_ref.astype(np.float64)) + 2 * k * uld * mag + 4 * k * U * U * mag
    err = np.abs(r_gpu - r_ref.astype(np.float64))
    assert np.all(err <= bound), float(np.max(err / bound))



def _residual_gpu(A, b, nu, lam, x):
    import ctypes

    from paper_2104_14101_amd import _binding as B

    n, d = A.shape
    c = b.shape[1]
    rd = torch.empty((d, c), dtype=torch.float64, device="cuda")
    At, bt, xt = to_dev(A), to_dev(b), to_dev(x)
    lt = to_dev(lam) if lam is not None else None
    h = aes._handle(torch.device("cuda:0"))
    st = B.load().aes_residual(h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), n, d, c,
                               ctypes.c_void_p(At.data_ptr()), d, ctypes.c_void_p(bt.data_ptr()), c, nu,
                               ctypes.c_void_p(lt.data_ptr() if lt is not None else 0),
                               ctypes.c_void_p(xt.data_ptr()), c, ctypes.c_void_p(rd.data_ptr()), c)
    assert st == B.AES_OK
    torch.cuda.synchronize()
    return rd.cpu().numpy()


@pytest.mark.parametrize("c", [1, 2, 8, 16, 32])
def test_compensated_residual_within_one_rounding_of_the_exact_value(c):
    # exact rational arithmetic on a small problem near its solution (the residual is ~1e-12 of
    # the terms it is the difference of): the compensated result is the exact residual rounded,
    # up to (n + d) u^2 of the terms' magnitude; the plain FP64 evaluation is not
    from fractions import Fraction

    rng = np.random.default_rng(5)
    n, d, nu = 200, 48, 1e-3
    A = rng.standard_normal((n, d)) * np.exp(-0.15 * np.arange(d))
    lam = 1.0 + rng.random(d)
    b = A.T @ rng.standard_normal((n, c))
    x = np.linalg.solve(A.T @ A + nu ** 2 * np.diag(lam), b)
    Af = [[Fraction(v) for v in row] for row in A]
    xf = [[Fraction(v) for v in row] for row in x]
    nu2 = Fraction(nu) ** 2
    r_exact = np.empty((d, c))
    for cc in range(c):
        z = [sum(Af[i][k] * xf[k][cc] for k in range(d)) for i in range(n)]
        for j in range(d):
            q = sum(Af[i][j] * z[i] for i in range(n)) + nu2 * Fraction(lam[j]) * xf[j][cc]
            r_exact[j, cc] = float(Fraction(b[j, cc]) - q)
    mag = np.abs(A).T @ (np.abs(A) @ np.abs(x)) + nu ** 2 * lam[:, None] * np.abs(x) + np.abs(b)
    bound = U * np.abs(r_exact) + 8 * (n + d) * U * U * mag
    r_gpu = _residual_gpu(A, b, nu, lam, x)
    assert np.all(np.abs(r_gpu - r_exact) <= bound), float(np.max(np.abs(r_gpu - r_exact) / bound))
    r_plain = b - A.T @ (A @ x) - nu ** 2 * lam[:, None] * x
    assert np.any(np.abs(r_plain - r_exact) > 100 * bound)
