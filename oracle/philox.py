"""Philox4x64-10 counter-based generator and the random streams drawn by the sketches.

Test infrastructure only (see ``oracle/__init__.py``).

Generator: Philox4x64 with 10 rounds, as published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  A 256-bit counter (c0..c3) and a
128-bit key (k0, k1) map to four 64-bit words.  Each round multiplies c0 and c2 by two fixed
odd constants, keeps the high and low halves of the 128-bit products, and mixes them with c1,
c3 and the key; the key is bumped by two Weyl constants between rounds.
Pin: ``numpy.random.Philox`` (an independent implementation of the same generator) in
tests/test_oracle_rng.py.

Random streams (a reading of the paper, which only says "random signs", "uniformly at random
without replacement" and "i.i.d. N(0, 1/m)" in Sec. 2.1):
  key     = (seed, (problem << 32) | k)      k = index of the sketch (0, 1, 2, ... per resize)
  SIGN    counter (i, 1, 0, 0): epsilon_i = -1 iff bit 63 of word 0 is set       (row i < n)
  ROW     counter (i, 2, 0, 0): 64-bit sort key of padded row i = word 0         (i < n')
  GAUSS   counter (i, 3, r >> 2, 0): the four words give four N(0,1) values for sketch rows
          4*(r>>2) .. 4*(r>>2)+3 of data column i, by the Box-Muller transform on the word
          pairs (w0, w1) and (w2, w3).
  SJLT    counter (i, 4, 0, 0): column i of S has its one non-zero in row
          h_i = floor(w0 * m / 2^64) (the high word of the 128-bit product, uniform on
          [0, m) up to m / 2^64), with value -1 iff bit 63 of w1 is set, else +1.
"""
import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

SIGN, ROW, GAUSS, SJLT = 1, 2, 3, 4


def _mulhilo(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps mod 2**64
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x64-`rounds` of counter arrays (broadcast together) under key (k0, k1).

    Returns four uint64 arrays.  Parity pinned against numpy.random.Philox.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for r in range(rounds):
            if r > 0:
                k0 = np.uint64(k0 + _W0)
                k1 = np.uint64(k1 + _W1)
            hi0, lo0 = _mulhilo(_M0, c0)
            hi1, lo1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def stream_key(seed, k, problem=0):
    """Key words for sketch number k of problem `problem` under the user seed."""
    return np.uint64(seed & 0xFFFFFFFFFFFFFFFF), np.uint64(((problem & 0xFFFFFFFF) << 32) | (k & 0xFFFFFFFF))


def signs(seed, k, n, problem=0):
    """Rademacher diagonal E of the SRHT for data rows 0..n-1 (float64 +-1)."""
    k0, k1 = stream_key(seed, k, problem)
    i = np.arange(n, dtype=np.uint64)
    w0, _, _, _ = philox4x64(i, SIGN, 0, 0, k0, k1)
    return np.where((w0 >> np.uint64(63)) != 0, -1.0, 1.0)


def row_keys(seed, k, npad, problem=0):
    """64-bit sort keys of the padded rows 0..npad-1; the SRHT keeps the m smallest."""
    k0, k1 = stream_key(seed, k, problem)
    i = np.arange(npad, dtype=np.uint64)
    w0, _, _, _ = philox4x64(i, ROW, 0, 0, k0, k1)
    return w0


def _u01_open0(w):
    """(w >> 11 + 1) * 2^-53, a uniform in (0, 1]."""
    return ((w >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def _u01(w):
    """(w >> 11) * 2^-53, a uniform in [0, 1)."""
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian_rows(seed, k, rows, i0, i1, problem=0):
    """N(0,1) block G[rows, i0:i1] of the Gaussian embedding before the 1/sqrt(m) scale.

    Box-Muller: z = sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).
    """
    rows = np.asarray(rows, dtype=np.int64)
    k0, k1 = stream_key(seed, k, problem)
    i = np.arange(i0, i1, dtype=np.uint64)[None, :]
    q = (rows >> 2).astype(np.uint64)[:, None]
    w0, w1, w2, w3 = philox4x64(i, GAUSS, q, 0, k0, k1)
    sel = (rows & 3)[:, None]
    first = sel < 2
    ua = np.where(first, _u01_open0(w0), _u01_open0(w2))
    ub = np.where(first, _u01(w1), _u01(w3))
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return np.where((sel & 1) == 0, rad * np.cos(ang), rad * np.sin(ang))


def sjlt_hash(seed, k, n, m, problem=0):
    """Row h_i in [0, m) and sign of the single non-zero of column i < n of an SJLT (s = 1)."""
    k0, k1 = stream_key(seed, k, problem)
    i = np.arange(n, dtype=np.uint64)
    w0, w1, _, _ = philox4x64(i, SJLT, 0, 0, k0, k1)
    with np.errstate(over="ignore"):
        hi, _ = _mulhilo(w0, np.full_like(w0, np.uint64(m)))
    sgn = np.where((w1 >> np.uint64(63)) != 0, -1.0, 1.0)
    return hi.astype(np.int64), sgn
