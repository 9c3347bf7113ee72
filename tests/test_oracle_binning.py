"""Pins of the oracle's quantile binning against closed forms and invariants."""
import numpy as np
import pytest

from oracle import oracle as O


def test_equal_frequency_on_distinct_values():
    # n = 37 * B distinct values: every bin holds exactly 37 values.
    for B in (4, 64, 256):
        n = 37 * B
        rng = np.random.default_rng(B)
        X = rng.permutation(n).astype(np.float32).reshape(n, 1) * 0.5 - 3.0
        bins, cuts, ncuts = O.bin_matrix(X, B)
        assert ncuts[0] == B - 1
        assert np.array_equal(np.bincount(bins[0], minlength=B), np.full(B, 37))
        # rank r value gets bin r // 37
        order = np.argsort(X[:, 0])
        assert np.array_equal(bins[0][order], np.arange(n) // 37)


def test_categorical_codes_keep_levels():
    rng = np.random.default_rng(3)
    for L in (2, 5, 16):
        X = rng.integers(0, L, size=(3000, 1)).astype(np.float32)
        bins, _, ncuts = O.bin_matrix(X, 256)
        # each level gets its own bin, in order: bin == code (the top level
        # may also appear as a cut, which no value lies above)
        assert L - 1 <= ncuts[0] <= L
        assert np.array_equal(bins[0], X[:, 0].astype(np.uint8))


def test_invariants_random():
    rng = np.random.default_rng(11)
    n, p = 777, 9
    X = rng.standard_normal((n, p)).astype(np.float32)
    X[:, 3] = np.round(X[:, 3] * 2)  # ties
    X[:, 4] = 1.5                   # constant column
    X[5, 5] = -0.0
    X[6, 5] = 0.0
    for B in (2, 16, 256):
        bins, cuts, ncuts = O.bin_matrix(X, B)
        for j in range(p):
            b = bins[j].astype(int)
            x = X[:, j]
            assert b.max() <= B - 1 and b.max() <= ncuts[j]
            o = np.argsort(x, kind="stable")
            assert np.all(np.diff(b[o]) >= 0)            # monotone in x
            for v in np.unique(x):
                assert len(set(b[x == v])) == 1           # equal values, equal bin
            assert ncuts[j] <= len(np.unique(x))
        assert np.all(bins[4] == 0)


def _numpy_definition(x, B):
    n = len(x)
    s = np.sort(x)
    ks = np.arange(1, B)
    ranks = -(-ks * n // B) - 1
    cand = s[ranks]
    uniq = [cand[0]]
    for c in cand[1:]:
        if c > uniq[-1]:
            uniq.append(c)
    return np.searchsorted(np.array(uniq, dtype=np.float32), x, side="left")


@pytest.mark.parametrize("B", [2, 3, 64, 255, 256])
def test_matches_numpy_definition(B):
    rng = np.random.default_rng(B + 100)
    for n in (2, 3, 50, 257, 1000):
        X = np.stack([rng.standard_normal(n), rng.integers(0, 7, n),
                      np.exp(rng.standard_normal(n))], axis=1).astype(np.float32)
        bins, _, _ = O.bin_matrix(X, B)
        for j in range(3):
            assert np.array_equal(bins[j], _numpy_definition(X[:, j], B))


def test_rejects_nonfinite():
    X = np.zeros((10, 2), np.float32)
    X[3, 1] = np.nan
    with pytest.raises(ValueError):
        O.bin_matrix(X, 8)
