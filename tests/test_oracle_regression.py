"""Pins of the oracle's regression forest (TreeImp): the split search against
an exhaustive brute force of the weighted squared-error definition with exact
rationals, against the classification oracle on the two-channel encoding that
the device uses, the target quantisation against numpy, and recovery of
planted features."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

Q = 255


def sse(rows, w, y):
    W = sum(int(w[i]) for i in rows)
    if W == 0:
        return Fraction(0)
    mean = Fraction(sum(int(w[i]) * int(y[i]) for i in rows), W)
    return sum(int(w[i]) * (int(y[i]) - mean) ** 2 for i in rows)


def brute_best_reg(bins, y, w, rows, feats, B):
    """Every (draw position, threshold) by its decrease of the weighted squared
    error; the first maximum in (position, threshold) order; split iff the
    decrease is strictly positive."""
    parent = sse(rows, w, y)
    best = None
    for q, f in enumerate(feats):
        for b in range(B - 1):
            left = [i for i in rows if bins[f][i] <= b]
            right = [i for i in rows if bins[f][i] > b]
            if not left or not right:
                continue
            d = parent - sse(left, w, y) - sse(right, w, y)
            if best is None or d > best[0]:
                best = (d, q, b, sum(int(w[i]) for i in left), sum(int(w[i]) for i in right))
    if best is None or not best[0] > 0:
        return None
    g = best[0] * 2**33 / Q
    return dict(q=best[1], b=best[2], nl=best[3], nr=best[4], gain_fix=g.numerator // g.denominator)


def test_split_search_is_the_squared_error_definition():
    rng = np.random.default_rng(21)
    for trial in range(250):
        n, p, B = int(rng.integers(2, 10)), int(rng.integers(1, 4)), int(rng.integers(2, 7))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        y = rng.integers(0, Q + 1, n).astype(np.int32)
        if trial % 5 == 0:
            y[:] = rng.integers(0, 3, n)  # many ties
        w = rng.integers(1, 4, n).astype(np.uint32)
        rows = np.arange(n, dtype=np.uint32)
        feats = rng.permutation(p)[: int(rng.integers(1, p + 1))].astype(np.int32)
        got = O.best_split_reg(bins, y, w, rows, feats, B)
        want = brute_best_reg(bins, y, w, rows, feats, B)
        if want is None:
            assert got["found"] == 0
        else:
            assert got["found"] == 1
            assert (got["q"], got["b"], got["nl"], got["nr"], got["gain_fix"]) == \
                (want["q"], want["b"], want["nl"], want["nr"], want["gain_fix"])


def test_two_channel_encoding_gives_the_same_split():
    # a row of level y and weight w as two class records (class 0 with weight
    # w (Q - y), class 1 with w y) under the Gini rule: same split, and a Gini
    # decrease floor(2^32 D_gini) equal to the regression floor(2^33 D / Q)
    rng = np.random.default_rng(22)
    for trial in range(150):
        n, p, B = int(rng.integers(2, 9)), int(rng.integers(1, 4)), int(rng.integers(2, 6))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        y = rng.integers(0, Q + 1, n).astype(np.int32)
        w = rng.integers(1, 3, n).astype(np.uint32)
        rows = np.arange(n, dtype=np.uint32)
        feats = rng.permutation(p).astype(np.int32)
        reg = O.best_split_reg(bins, y, w, rows, feats, B)
        bins2 = np.concatenate([bins, bins], axis=1)
        y2 = np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)])
        w2 = np.concatenate([w * (Q - y), w * y]).astype(np.uint32)
        rows2 = np.flatnonzero(w2).astype(np.uint32)
        cls = O.best_split(bins2, y2, w2, rows2, feats, 2, B)
        assert cls["found"] == reg["found"]
        if reg["found"]:
            assert (cls["q"], cls["b"], cls["gain_fix"]) == (reg["q"], reg["b"], reg["gain_fix"])
            assert (cls["nl"], cls["nr"]) == (Q * reg["nl"], Q * reg["nr"])


def test_target_quantisation_matches_numpy():
    rng = np.random.default_rng(23)
    for scale in (1e-3, 1.0, 7.5e4):
        y = (rng.standard_normal(1000) * scale).astype(np.float32)
        y64 = y.astype(np.float64)
        lo, hi = y64.min(), y64.max()
        want = np.floor((y64 - lo) * Q / (hi - lo) + 0.5).astype(np.int32)
        got = O.quantize_target(y)
        assert np.array_equal(got, want)
        assert got.min() == 0 and got.max() == Q
    assert not O.quantize_target(np.full(10, 3.25, np.float32)).any()


def test_planted_regression_features_recovered():
    rng = np.random.default_rng(24)
    n, p = 600, 12
    X = rng.random((n, p)).astype(np.float32)
    y = (4 * X[:, 0] + 3 * np.sin(3 * X[:, 1]) + 2 * (X[:, 2] > 0.5)
         + 0.3 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, 40, 8, max_iter=30, seed=5, n_bins=64)
    assert list(r["decision"][:3]) == [1, 1, 1]
    assert (r["decision"][3:] <= 0).all()
    assert (r["decision"][3:] == -1).sum() >= 6
    assert list(r["rank"][:3]) == [1, 1, 1]


def test_regression_arguments_checked():
    X = np.zeros((10, 3), np.float32)
    with pytest.raises(ValueError):
        O.boruta_fit_reg(X, np.arange(10, dtype=np.float32), 2, 2, importance_mode=3)
    y = np.arange(10, dtype=np.float32)
    y[3] = np.inf
    with pytest.raises(ValueError):
        O.boruta_fit_reg(X, y, 2, 2)


def test_permutation_importance_of_stumps_recomputed_in_python():
    # Permut for regression on depth-1 trees, recomputed here from the
    # definition: leaf mean level floor(256 T / W) of the in-bag rows on each
    # side of the root split, squared errors in 1/65536 level^2 units, and the
    # OOB rows' error increase when the root column's bins are moved by the
    # keyed permutation of the OOB set (shadow columns rebuilt by their own
    # keyed row permutation)
    rng = np.random.default_rng(25)
    n, p, B, T, R, seed = 400, 6, 16, 7, 2, 9
    X = rng.random((n, p)).astype(np.float32)
    y = (3 * X[:, 0] + np.sin(5 * X[:, 1]) + 0.3 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, T, 1, importance_mode=1, max_iter=1, seed=seed, n_bins=B,
                         n_perm=R, trace=True)
    tr = r["traces"][0]
    bins, _, _ = O.bin_matrix(X, B)
    yq = O.quantize_target(y).astype(np.int64)
    p_cur = tr["p_cur"]

    def column(fw):
        src = tr["col_src"][fw]
        if fw < p_cur:
            return bins[src]
        s = fw - p_cur
        return np.array([bins[src][O.keyed_perm(seed, 3, 1, s, 0, 0, n, i)] for i in range(n)])

    want = np.zeros(tr["p_w"], np.int64)
    for tau in range(T):
        w = O.bootstrap(seed, 1, tau, n).astype(np.int64)
        root = tr["nodes"][(tr["nodes"][:, 0] == tau) & (tr["nodes"][:, 1] == 1)][0]
        f, b = int(root[2]), int(root[3])
        if f < 0:
            continue
        col = column(f).astype(np.int64)
        left = col <= b
        v = {}
        for side in (True, False):
            m_in = (w > 0) & (left == side)
            v[side] = (256 * int((w[m_in] * yq[m_in]).sum())) // int(w[m_in].sum())
        oob = np.flatnonzero(w == 0)
        m = len(oob)
        for rep in range(R):
            for j in range(m):
                src = O.keyed_perm(seed, 4, 1, tau, f, rep << 16, m, j)
                e1 = v[bool(col[oob[src]] <= b)] - 256 * yq[oob[j]]
                e0 = v[bool(col[oob[j]] <= b)] - 256 * yq[oob[j]]
                want[f] += e1 * e1 - e0 * e0
    assert np.array_equal(tr["imp_int"], want)
    assert want[0] > 0


def test_permutation_importance_path_restricted_equals_naive():
    X, y = _problem(26)
    kw = dict(importance_mode=1, max_iter=4, seed=2, n_bins=32, n_perm=2, trace=True)
    a = O.boruta_fit_reg(X, y, 6, 7, **kw)
    b = O.boruta_fit_reg(X, y, 6, 7, permut_naive=True, **kw)
    assert np.array_equal(a["decision"], b["decision"])
    for ta, tb in zip(a["traces"], b["traces"]):
        assert np.array_equal(ta["imp_int"], tb["imp_int"])
        # a column no tree splits on has exactly zero importance
        used = np.unique(ta["nodes"][ta["nodes"][:, 2] >= 0, 2])
        assert not ta["imp_int"][np.setdiff1d(np.arange(ta["p_w"]), used)].any()


def test_planted_regression_features_recovered_by_permutation():
    X, y = _problem(27)
    r = O.boruta_fit_reg(X, y, 40, 8, importance_mode=1, max_iter=30, seed=5, n_bins=64)
    assert list(r["decision"][:3]) == [1, 1, 1]
    assert (r["decision"][3:] == -1).sum() >= 6


def _problem(seed, n=600, p=12):
    rng = np.random.default_rng(seed)
    X = rng.random((n, p)).astype(np.float32)
    y = (4 * X[:, 0] + 3 * np.sin(3 * X[:, 1]) + 2 * (X[:, 2] > 0.5)
         + 0.3 * rng.standard_normal(n)).astype(np.float32)
    return X, y


def test_divergence_importance_of_stumps_recomputed_in_python():
    # Algorithm 3 for regression on depth-1 trees, recomputed here: the shared
    # row permutation of the iteration, per row the change D of the summed
    # leaf levels floor(256 T / W) when the column is permuted, and the sum
    # over rows of floor(D^2 / T^2)
    rng = np.random.default_rng(28)
    n, p, B, T, seed = 300, 5, 16, 6, 4
    X = rng.random((n, p)).astype(np.float32)
    y = (3 * X[:, 0] + np.sin(5 * X[:, 1]) + 0.3 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, T, 1, importance_mode=2, max_iter=1, seed=seed, n_bins=B,
                         trace=True)
    tr = r["traces"][0]
    bins, _, _ = O.bin_matrix(X, B)
    yq = O.quantize_target(y).astype(np.int64)
    p_cur = tr["p_cur"]

    def column(fw):
        src = tr["col_src"][fw]
        if fw < p_cur:
            return bins[src].astype(np.int64)
        s = fw - p_cur
        return np.array([bins[src][O.keyed_perm(seed, 3, 1, s, 0, 0, n, i)] for i in range(n)],
                        np.int64)

    pi = np.array([O.keyed_perm(seed, 5, 1, 0, 0, 0, n, i) for i in range(n)])
    stumps = []
    for tau in range(T):
        w = O.bootstrap(seed, 1, tau, n).astype(np.int64)
        root = tr["nodes"][(tr["nodes"][:, 0] == tau) & (tr["nodes"][:, 1] == 1)][0]
        f, b = int(root[2]), int(root[3])
        if f < 0:
            continue
        col = column(f)
        v = {}
        for side in (True, False):
            m_in = (w > 0) & ((col <= b) == side)
            v[side] = (256 * int((w[m_in] * yq[m_in]).sum())) // int(w[m_in].sum())
        stumps.append((f, b, col, v))
    want = np.zeros(tr["p_w"], np.int64)
    for f in range(tr["p_w"]):
        for row in range(n):
            d = 0
            for (g, b, col, v) in stumps:
                if g == f:
                    d += v[bool(col[pi[row]] <= b)] - v[bool(col[row] <= b)]
            want[f] += (d * d) // (T * T)
    assert np.array_equal(tr["imp_int"], want)
    assert want[0] > 0
