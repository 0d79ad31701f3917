"""Pins of the oracle's Philox4x64-10 and of the random streams it derives."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 123456789), (0xDEADBEEF, 2**40 + 3)])
@pytest.mark.parametrize("start", [0, 1, 1000, 2**63 + 17])
def test_philox_matches_numpy(key, start):
    # numpy's Philox increments its 256-bit counter before producing each block of 4 words.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([start, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(4 * 6).reshape(6, 4)
    ctr = (np.arange(6, dtype=np.uint64) + np.uint64(start) + np.uint64(1))
    w = philox.philox4x64(ctr, 0, 0, 0, key[0], key[1])
    np.testing.assert_array_equal(np.stack(w, axis=1), raw)


def test_philox_high_counter_words_match_numpy():
    c = np.array([2**64 - 1, 5, 9, 11], dtype=np.uint64)  # increment carries into word 1
    bg = np.random.Philox(key=np.array([3, 4], dtype=np.uint64), counter=c)
    raw = bg.random_raw(4)
    w = philox.philox4x64(0, 6, 9, 11, 3, 4)
    np.testing.assert_array_equal(np.array([int(v) for v in w], dtype=np.uint64), raw)


def test_signs_balanced_and_keyed():
    e = philox.signs(1, 0, 200000)
    assert set(np.unique(e)) == {-1.0, 1.0}
    assert abs(e.mean()) < 5 * (1 / np.sqrt(len(e)))
    e2 = philox.signs(1, 1, 200000)
    assert np.mean(e == e2) < 0.52  # fresh randomness per sketch index
    e3 = philox.signs(1, 0, 200000, problem=1)
    assert np.mean(e == e3) < 0.52


def test_gaussian_moments():
    G = philox.gaussian_rows(3, 0, np.arange(64), 0, 4096)
    z = G.ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # rows within one counter block are independent (pairwise correlation ~ 0)
    c = np.corrcoef(G[:4])
    assert np.max(np.abs(c - np.eye(4))) < 0.06


def test_gaussian_block_consistency():
    full = philox.gaussian_rows(9, 2, np.arange(10), 0, 300)
    part = philox.gaussian_rows(9, 2, np.array([3, 7]), 100, 200)
    np.testing.assert_array_equal(full[[3, 7], 100:200], part)
