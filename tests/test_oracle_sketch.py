"""Pins of the oracle's SRHT and Gaussian embeddings (Sec. 2.1)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import philox
from oracle import sketch as sk


@pytest.mark.parametrize("n", [1, 2, 8, 64, 1024])
def test_fwht_equals_sylvester_hadamard(n):
    X = np.random.default_rng(n).standard_normal((n, 5))
    np.testing.assert_allclose(sk.fwht_rows(X), sla.hadamard(n) @ X, rtol=0, atol=1e-12 * n)


def test_fwht_orthogonality_and_symmetry():
    n = 256
    H = sk.fwht_rows(np.eye(n))
    np.testing.assert_array_equal(H, H.T)
    np.testing.assert_array_equal(H @ H, n * np.eye(n))


def test_fwht_bit_exact_on_integers():
    n = 512
    X = np.random.default_rng(0).integers(-1000, 1000, size=(n, 7)).astype(np.float64)
    np.testing.assert_array_equal(sk.fwht_rows(X), (sla.hadamard(n).astype(np.int64) @ X.astype(np.int64)).astype(np.float64))


def test_padded_size():
    assert [sk.padded_size(v) for v in (1, 2, 3, 4, 5, 4096, 4097)] == [1, 2, 4, 4, 8, 4096, 8192]


def test_srht_full_size_is_isometry():
    # m = n' => S^T S = I_n' (the normalised Hadamard is orthogonal), so (SA)^T SA = A^T A.
    rng = np.random.default_rng(1)
    A = rng.standard_normal((100, 6))  # n' = 128: padding exercised
    SA = sk.srht(A, 128, seed=4, k=0)
    np.testing.assert_allclose(SA.T @ SA, A.T @ A, rtol=1e-12, atol=1e-12)


def test_srht_matrix_form_and_rows():
    rng = np.random.default_rng(2)
    n, d, m = 37, 4, 9
    A = rng.standard_normal((n, d))
    SA = sk.srht(A, m, seed=11, k=3)
    R = sk.srht_rows(11, 3, n, m)
    assert len(set(R.tolist())) == m and np.all(np.diff(R) > 0) and R.max() < 64
    eps = philox.signs(11, 3, n)
    Hn = sla.hadamard(64)[R][:, :n]
    S = Hn * eps[None, :] / np.sqrt(m)
    np.testing.assert_allclose(SA, S @ A, rtol=1e-13, atol=1e-13)
    for j in (0, 4, 8):
        np.testing.assert_allclose(sk.srht_row(A, m, 11, 3, j), SA[j], rtol=1e-13, atol=1e-13)


def test_srht_reuse_matrix_form():
    # S_k = H[R_k] E_0 / sqrt(m): rows of sketch index k, signs of index 0 (a sign draw keyed by
    # k, or rows keyed by 0, fails this)
    rng = np.random.default_rng(3)
    n, d, m = 37, 4, 9
    A = rng.standard_normal((n, d))
    for k in (1, 3):
        SA = sk.srht_reuse(A, m, seed=11, k=k)
        R = sk.srht_rows(11, k, n, m)
        eps0 = philox.signs(11, 0, n)
        S = sla.hadamard(64)[R][:, :n] * eps0[None, :] / np.sqrt(m)
        np.testing.assert_allclose(SA, S @ A, rtol=1e-13, atol=1e-13)
    # index 0 is the SRHT of index 0; m = n' is an isometry for every k
    np.testing.assert_allclose(sk.srht_reuse(A, m, 11, 0), sk.srht(A, m, 11, 0), rtol=1e-14, atol=1e-14)
    SA = sk.srht_reuse(A, 64, 11, 5)
    np.testing.assert_allclose(SA.T @ SA, A.T @ A, rtol=1e-12, atol=1e-12)


def test_srht_nested_rows_and_prefixes():
    # the rows of size m are the SRHT sample of index 0 (same rows, same scale), listed in key
    # order; size m is the first m rows of size 2m up to the scale sqrt(n'/m)
    rng = np.random.default_rng(8)
    n, d = 45, 5
    A = rng.standard_normal((n, d))
    npad = sk.padded_size(n)
    keys = philox.row_keys(13, 0, npad)
    for m in (1, 4, 7, 16, 64):
        R = sk.srht_nested_rows(13, n, m)
        np.testing.assert_array_equal(np.sort(R), sk.srht_rows(13, 0, n, m))
        assert np.all(np.diff(keys[R].astype(object)) > 0)
        SA = sk.srht_nested(A, m, 13)
        np.testing.assert_allclose(SA[np.argsort(R)], sk.srht(A, m, 13, 0), rtol=1e-13, atol=1e-13)
    for m in (1, 3, 8, 32):
        big = sk.srht_nested(A, 2 * m, 13)
        np.testing.assert_allclose(sk.srht_nested(A, m, 13) * np.sqrt(m), big[:m] * np.sqrt(2 * m),
                                   rtol=1e-14, atol=1e-14)
    # the sketch index plays no part; m = n' is an isometry
    np.testing.assert_array_equal(sk.sketch(A, 8, "srht_nested", 13, 0), sk.sketch(A, 8, "srht_nested", 13, 5))
    SA = sk.srht_nested(A, npad, 13)
    np.testing.assert_allclose(SA.T @ SA, A.T @ A, rtol=1e-12, atol=1e-12)


def test_srht_nested_incremental_gram():
    # (S_m' A)^T S_m' A = (m/m') (S_m A)^T S_m A + Gram of the rows m..m'-1 of S_m' A, for the
    # doubling step and an uneven one (a capped last resize)
    rng = np.random.default_rng(9)
    n, d = 100, 6
    A = rng.standard_normal((n, d))
    for m, m2 in ((8, 16), (16, 32), (24, 128), (32, 40)):
        G_small = sk.srht_nested(A, m, 2).T @ sk.srht_nested(A, m, 2)
        big = sk.srht_nested(A, m2, 2)
        inc = (m / m2) * G_small + big[m:].T @ big[m:]
        np.testing.assert_allclose(inc, big.T @ big, rtol=1e-12, atol=1e-12)
    # with the old rows re-weighted by 1/2 instead of m/m' the identity fails for m' = 5m/4
    big = sk.srht_nested(A, 40, 2)
    G32 = sk.srht_nested(A, 32, 2).T @ sk.srht_nested(A, 32, 2)
    assert np.max(np.abs(0.5 * G32 + big[32:].T @ big[32:] - big.T @ big)) > 1e-3


def test_srht_nested_unbiased_over_seeds():
    # E[S_m^T S_m] = I over the seed (the sketch index is fixed for this variant)
    n, m, reps = 16, 4, 600
    acc = np.zeros((n, n))
    for seed in range(reps):
        SA = sk.srht_nested(np.eye(n), m, seed)
        acc += SA.T @ SA
    acc /= reps
    assert np.max(np.abs(acc - np.eye(n))) < 0.25
    assert abs(np.trace(acc) / n - 1) < 0.05


def _sts(kind, n, m, seed, k):
    return np.array(sk.sketch(np.eye(n), m, kind, seed, k)).T @ np.array(sk.sketch(np.eye(n), m, kind, seed, k))


@pytest.mark.parametrize("kind", ["srht", "gauss", "sjlt", "srht_reuse"])
def test_sketch_unbiased(kind):
    # E[S^T S] = I: average over independent sketch indices (Monte Carlo).
    n, m, reps = 16, 4, 600
    acc = np.zeros((n, n))
    for k in range(reps):
        SA = sk.sketch(np.eye(n), m, kind, seed=5, k=k)
        acc += SA.T @ SA
    acc /= reps
    assert np.max(np.abs(acc - np.eye(n))) < 0.25
    assert abs(np.trace(acc) / n - 1) < 0.05


def test_srht_row_sample_uniform():
    npad, m, reps = 32, 8, 4000
    counts = np.zeros(npad)
    for k in range(reps):
        counts[sk.srht_rows(7, k, npad, m)] += 1
    expected = reps * m / npad
    chi2 = np.sum((counts - expected) ** 2 / expected)
    from scipy import stats
    assert stats.chi2.sf(chi2, npad - 1) > 1e-4


def test_gaussian_sketch_matches_definition():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((50, 3))
    SA = sk.gaussian(A, 6, seed=2, k=1, chunk=16)
    G = philox.gaussian_rows(2, 1, np.arange(6), 0, 50)
    np.testing.assert_allclose(SA, G @ A / np.sqrt(6), rtol=1e-13, atol=1e-13)


def test_gaussian_embedding_theorem_statistical():
    # Gaussian concentration theorem: with m >= (sqrt(d_e) + sqrt(8 log(16/delta)))^2 / rho,
    # eig(C_S - I) lies in ||D||^2 (-2 sqrt(rho) + rho, 2 sqrt(rho) + rho) w.p. >= 1 - delta.
    from oracle.factor import SketchedHessian
    rng = np.random.default_rng(4)
    n, d, nu, rho, delta = 256, 6, 0.3, 0.5, 0.5
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    sig = 0.7 ** np.arange(1, d + 1)
    A = U * sig
    H = A.T @ A + nu ** 2 * np.eye(d)
    D2 = sig ** 2 / (sig ** 2 + nu ** 2)
    de = D2.sum() / D2.max()
    m = int(np.ceil((np.sqrt(de) + np.sqrt(8 * np.log(16 / delta))) ** 2 / rho))
    w, V = np.linalg.eigh(H)
    Hm12 = V @ np.diag(w ** -0.5) @ V.T
    ok = 0
    reps = 40
    for k in range(reps):
        HS = SketchedHessian(sk.gaussian(A, m, seed=8, k=k), nu, np.ones(d)).matrix()
        ev = np.linalg.eigvalsh(Hm12 @ HS @ Hm12 - np.eye(d))
        ok += (ev.min() >= D2.max() * (-2 * np.sqrt(rho) + rho)) and (ev.max() <= D2.max() * (2 * np.sqrt(rho) + rho))
    assert ok / reps >= 1 - delta


def test_sjlt_is_one_signed_entry_per_column():
    # S built densely from the hash: one +-1 per column, S A by a dense product, and the
    # bucket map equal to the high word of w0 * m in Python big-integer arithmetic.
    n, m, d = 37, 5, 3
    h, sgn = philox.sjlt_hash(11, 2, n, m)
    k0, k1 = philox.stream_key(11, 2)
    w0, w1, _, _ = philox.philox4x64(np.arange(n, dtype=np.uint64), philox.SJLT, 0, 0, k0, k1)
    assert [int(v) for v in h] == [(int(a) * m) >> 64 for a in w0]
    assert [float(v) for v in sgn] == [-1.0 if int(b) >> 63 else 1.0 for b in w1]
    S = np.zeros((m, n))
    S[h, np.arange(n)] = sgn
    assert np.all(np.count_nonzero(S, axis=0) == 1) and set(np.unique(S)) <= {-1.0, 0.0, 1.0}
    np.testing.assert_array_equal(np.diag(S.T @ S), np.ones(n))
    A = np.random.default_rng(5).integers(-50, 50, size=(n, d)).astype(np.float64)
    np.testing.assert_array_equal(sk.sjlt(A, m, 11, 2), S @ A)  # integers: exact


def test_sjlt_sums_in_row_order():
    # a small value followed by two opposite huge ones in one bucket: summed left to right
    # from zero the small one is absorbed (0.0); any order that cancels the huge pair first
    # would give 1.0
    n = 40
    h, sgn = philox.sjlt_hash(3, 0, n, 1)
    A = np.zeros((n, 1))
    A[0, 0], A[1, 0], A[2, 0] = 1.0 * sgn[0], 1e16 * sgn[1], -1e16 * sgn[2]
    assert sk.sjlt(A, 1, 3, 0)[0, 0] == 0.0


def test_sjlt_buckets_and_signs_uniform():
    from scipy import stats
    n, m = 200000, 7
    h, sgn = philox.sjlt_hash(9, 4, n, m)
    assert h.min() >= 0 and h.max() < m
    counts = np.bincount(h, minlength=m)
    expected = n / m
    assert stats.chi2.sf(np.sum((counts - expected) ** 2 / expected), m - 1) > 1e-4
    assert abs(sgn.mean()) < 5 / np.sqrt(n)


def test_sjlt_second_moment_closed_form():
    # M = U^T S^T S U - I = sum_{i != j} s_i s_j [h_i = h_j] u_i u_j^T, so for i.i.d. uniform
    # buckets and signs E||M||_F^2 = (d^2 + d - 2 sum_i ||u_i||^4) / m.
    rng = np.random.default_rng(8)
    n, d, m, reps = 300, 4, 32, 400
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    expect = (d * d + d - 2 * np.sum(np.sum(U * U, axis=1) ** 2)) / m
    vals = []
    for k in range(reps):
        SU = sk.sjlt(U, m, 21, k)
        vals.append(np.sum((SU.T @ SU - np.eye(d)) ** 2))
    vals = np.array(vals)
    assert abs(vals.mean() - expect) < 4 * vals.std() / np.sqrt(reps)
