"""Random embeddings S and the sketch S·A.  Test infrastructure only.

SRHT (Sec. 2.1 and the SRHT concentration proof): S = R H E, with E a diagonal of random
signs, H the Walsh-Hadamard matrix of the zero-padded size n' = 2^ceil(log2 n) (footnote of
Sec. 2.1: pad A with zero rows), and R a uniform row subsample without replacement.  The
proof section uses the normalised transform and the analysis scales by sqrt(n/m); this
oracle therefore forms

    S A = sqrt(n'/m) * R * (H_unnorm / sqrt(n')) * E * A_pad = (1/sqrt(m)) * R * H_unnorm * E * A_pad,

so that E[S^T S] = I (reading of the scale; with m = n' it gives S^T S = I exactly).
H_unnorm[i, j] = (-1)^popcount(i & j) is the Sylvester (natural) ordering.

Gaussian (Sec. 2.1): S has i.i.d. N(0, 1/m) entries, S = G / sqrt(m).

SJLT with s = 1 (Sec. 2.1): every column of S has exactly one non-zero, in a uniformly random
row, equal to +-1 with equal probability (1/sqrt(s) = 1), so S^T S has a unit diagonal and
E[S^T S] = I; S A adds each signed row of A into its row of the sketch.

Pins (tests/test_oracle_sketch.py): FWHT == scipy.linalg.hadamard(n') @ X, H^2 = n' I,
bit-exact on integer data; m = n' SRHT gives (SA)^T SA = A^T A; Monte-Carlo E[S^T S] = I for
the three embeddings; uniform marginals of the row sample; Gaussian moments; the SJLT as a dense
S with one +-1 per column, its hash against big-integer arithmetic, uniform buckets and the
closed-form second moment of U^T S^T S U - I; for ``srht_reuse``: its dense matrix form
from scipy's Hadamard matrix with the signs of index 0, equality with the SRHT at k = 0, the
isometry at m = n' and the Monte-Carlo mean over k of S_k^T S_k with E_0 fixed; for
``srht_nested``: its rows as a reordering of the SRHT of index 0, the prefix property, keys in
increasing order, the incremental Gram identity and the Monte-Carlo mean over seeds.
"""
import numpy as np

from . import philox


def padded_size(n):
    """n' = 2^ceil(log2 n), the Hadamard size after zero padding."""
    n = int(n)
    return 1 if n <= 1 else 1 << (n - 1).bit_length()


def fwht_rows(X):
    """Unnormalised Walsh-Hadamard transform along axis 0 (length must be a power of two).

    Radix-2 butterflies, one stage per bit of the row index: (a, b) -> (a + b, a - b).
    """
    Y = np.array(X, dtype=np.float64, copy=True)
    n = Y.shape[0]
    assert n & (n - 1) == 0, "FWHT length must be a power of two"
    rest = Y.shape[1:]
    h = 1
    while h < n:
        Z = Y.reshape((n // (2 * h), 2, h) + rest)  # a view: writes land in Y
        a = Z[:, 0].copy()
        b = Z[:, 1].copy()
        Z[:, 0] = a + b
        Z[:, 1] = a - b
        h *= 2
    return Y


def srht_rows(seed, k, n, m, problem=0):
    """Sorted indices R (length m) of the padded rows the SRHT keeps.

    The m padded rows with the smallest Philox ROW keys, ties broken by the smaller index
    (a uniform sample without replacement), listed in increasing row order.
    """
    npad = padded_size(n)
    if not 1 <= m <= npad:
        raise ValueError("SRHT sketch size must lie in [1, n']")
    keys = philox.row_keys(seed, k, npad, problem)
    order = np.argsort(keys, kind="stable")  # stable: equal keys keep increasing index
    return np.sort(order[:m])


def srht(A, m, seed, k, problem=0):
    """S A for an SRHT of size m x n (Sec. 2.1); A is n x d, returns m x d float64."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    npad = padded_size(n)
    eps = philox.signs(seed, k, n, problem)
    X = np.zeros((npad, d))
    X[:n] = eps[:, None] * A
    Y = fwht_rows(X)
    R = srht_rows(seed, k, n, m, problem)
    return Y[R] / np.sqrt(m)


def srht_reuse(A, m, seed, k, problem=0):
    """S_k A for the transform-reuse variant of the SRHT (not the paper's method).

    S_k = sqrt(n'/m) R_k (H / sqrt(n')) E_0: the signs of sketch index 0 for every k, the row
    sample R_k of index k.  Each S_k on its own is an SRHT, so a bound that holds for one SRHT
    holds for every S_k (a union bound over the resizes still applies), but the S_k share E_0
    and are not independent.  Computed from the normalised transform of A itself,
    Y = (H / sqrt(n')) E_0 A_pad (the SRHT of index 0 at m = n', which keeps every row in
    order), as sqrt(n'/m) Y[R_k]: the transform is the same for every resize.
    """
    A = np.asarray(A, dtype=np.float64)
    npad = padded_size(A.shape[0])
    Y = srht(A, npad, seed, 0, problem)
    R = srht_rows(seed, k, A.shape[0], m, problem)
    return Y[R] * np.sqrt(npad / m)


def srht_nested_rows(seed, n, m, problem=0):
    """Indices of the padded rows of the nested SRHT of size m, in the order they are listed.

    The m padded rows with the smallest Philox ROW keys of sketch index 0 (the sample rule of
    ``srht_rows``), listed in increasing key order with ties broken by the smaller index, so
    that the rows of size m are the first m of every larger size.
    """
    npad = padded_size(n)
    if not 1 <= m <= npad:
        raise ValueError("SRHT sketch size must lie in [1, n']")
    keys = philox.row_keys(seed, 0, npad, problem)
    return np.argsort(keys, kind="stable")[:m]


def srht_nested(A, m, seed, problem=0):
    """S_m A for the nested variant of the transform-reuse SRHT (not the paper's method).

    S_m = sqrt(n'/m) R_m (H / sqrt(n')) E_0 with R_m the first m rows of one random order of the
    n' padded rows (``srht_nested_rows``): every resize keeps the rows it had and adds new ones.
    Each S_m on its own is the SRHT of index 0 with its rows reordered, so a bound that holds
    for one SRHT holds for every S_m (a union bound over the resizes applies).  Its Gram then
    grows incrementally: with Y the normalised transform and m' > m,
    (S_m' A)^T S_m' A = (m/m') (S_m A)^T S_m A + (n'/m') sum over the new rows of y y^T.
    The sketch does not depend on a sketch index.
    """
    A = np.asarray(A, dtype=np.float64)
    npad = padded_size(A.shape[0])
    Y = srht(A, npad, seed, 0, problem)  # every padded row, in order: Y = (H / sqrt(n')) E_0 A_pad
    R = srht_nested_rows(seed, A.shape[0], m, problem)
    return Y[R] * np.sqrt(npad / m)


def srht_row(A, m, seed, k, j, problem=0):
    """Row j of S A computed directly from H's closed form, for spot checks at large n."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    R = srht_rows(seed, k, n, m, problem)
    i = np.int64(R[j])
    eps = philox.signs(seed, k, n, problem)
    rows = np.arange(n, dtype=np.int64)
    par = np.array([bin(int(v)).count("1") & 1 for v in (rows & i)], dtype=np.int64)
    h = np.where(par == 0, 1.0, -1.0)
    return (h * eps) @ A / np.sqrt(m)


def gaussian(A, m, seed, k, problem=0, chunk=4096):
    """S A for a Gaussian embedding with N(0, 1/m) entries (Sec. 2.1); O(m n d)."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    out = np.zeros((m, d))
    for r0 in range(0, m, 256):
        rows = np.arange(r0, min(m, r0 + 256))
        acc = np.zeros((len(rows), d))
        for i0 in range(0, n, chunk):
            i1 = min(n, i0 + chunk)
            G = gaussian_cols(seed, k, rows, i0, i1, problem)
            acc += G @ A[i0:i1]
        out[rows] = acc
    return out / np.sqrt(m)


def sjlt(A, m, seed, k, problem=0):
    """S A for an SJLT with s = 1 of size m x n (Sec. 2.1); A is n x d, returns m x d float64.

    Row r of S A is the sum, in increasing data-row order starting from zero, of sigma_i A_i
    over the rows i hashed to r.
    """
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    if m < 1:
        raise ValueError("SJLT sketch size must be positive")
    h, sgn = philox.sjlt_hash(seed, k, n, m, problem)
    out = np.zeros((m, d))
    np.add.at(out, h, sgn[:, None] * A)  # unbuffered: applied row by row in order of i
    return out


def gaussian_cols(seed, k, rows, i0, i1, problem=0):
    """Block G[rows, i0:i1] of the unscaled Gaussian matrix."""
    return philox.gaussian_rows(seed, k, rows, i0, i1, problem)


def sketch(A, m, kind, seed, k, problem=0):
    if kind == "srht":
        return srht(A, m, seed, k, problem)
    if kind == "srht_reuse":
        return srht_reuse(A, m, seed, k, problem)
    if kind == "srht_nested":
        return srht_nested(A, m, seed, problem)
    if kind == "gauss":
        return gaussian(A, m, seed, k, problem)
    if kind == "sjlt":
        return sjlt(A, m, seed, k, problem)
    raise ValueError(f"unknown sketch kind {kind!r}")


def max_sketch_size(n, kind):
    """Largest m the adaptive loop may reach: n' for both embeddings (cap reading)."""
    return padded_size(n)
