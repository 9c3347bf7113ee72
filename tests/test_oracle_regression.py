"""Pins of the oracle's regression forest (the paper's regression experiments
run Boruta on a random-forest regressor with squared-error loss, Sec. 2.2 and
Sec. 3): targets held exactly as 64-bit fixed point, the split search against
an exhaustive brute force over the float32 targets' exact rational values
(Fractions), against scikit-learn's regression tree at the root, the
fixed-point shifts against the bounds they must keep, Permut and Algorithm 3
recomputed in Python from their definitions on depth-1 forests, naive vs
path-restricted Permut, and recovery of planted features (also past 65,536
rows)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def exact(v):
    return Fraction(float(v))


def sse(rows, w, y):
    W = sum(int(w[i]) for i in rows)
    if W == 0:
        return Fraction(0)
    mean = sum(int(w[i]) * exact(y[i]) for i in rows) / W
    return sum(int(w[i]) * (exact(y[i]) - mean) ** 2 for i in rows)


def brute_best_reg(bins, y, w, rows, feats, B):
    """Every (draw position, threshold) by its decrease of the weighted squared
    error of the float targets (exact rationals); the first maximum in
    (position, threshold) order; split iff the decrease is strictly positive.
    Returns the decrease as a Fraction in target units."""
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
    return dict(d=best[0], q=best[1], b=best[2], wl=best[3], wr=best[4])


def exact_targets(rng, n, ties=False):
    """float32 targets within 15 binades of their largest magnitude, so that
    the fixed point holds them exactly: multiples of 1/8 in [-50, 50] with
    random extra low bits, or a few repeated values."""
    if ties:
        return rng.choice(np.float32([-1.25, 0.5, 3.0]), n).astype(np.float32)
    base = rng.integers(-400, 401, n).astype(np.float64) / 8.0
    return (base + rng.integers(0, 2 ** 8, n) / 2.0 ** 14).astype(np.float32)


def test_fixed_point_targets_are_exact():
    rng = np.random.default_rng(20)
    for scale in (1e-30, 1e-3, 1.0, 7.5e4, 3e30):
        y = (rng.standard_normal(2000) * scale).astype(np.float32)
        yfix, e, sh = O.fix_targets(y)
        m = np.abs(y.astype(np.float64)).max()
        assert m < 2.0 ** e <= 2 * m  # e is the smallest power above the maximum
        assert np.abs(yfix).max() < 2 ** 38
        assert np.abs(yfix).max() >= 2 ** 37
        # exact for every target of magnitude at least 2^(e - 15)
        big = np.abs(y.astype(np.float64)) >= 2.0 ** (e - 15)
        back = [Fraction(int(v)) * Fraction(2) ** (e - 38) for v in yfix[big][:300]]
        assert back == [exact(v) for v in y[big][:300]]
        # the others within half a unit of 2^(e - 38)
        for v, f in zip(y[~big][:200], yfix[~big][:200]):
            assert abs(exact(v) - Fraction(int(f)) * Fraction(2) ** (e - 38)) <= \
                Fraction(2) ** (e - 39)
        assert sh["range"] == int(yfix.max()) - int(yfix.min())
    z, e, sh = O.fix_targets(np.zeros(5, np.float32))
    assert not z.any() and sh["range"] == 0 and sh["s_gain"] == 0


def test_shifts_keep_the_sums_within_64_bits():
    # a tree's summed decrease <= n R^2 / 4 (R the fixed-point range) must stay
    # below 2^62 after the gain shift; the Permut sums (n_trees n_perm n terms
    # of at most (R + 1)^2) and the divergence sums (n terms of at most
    # (R + 1)^2) below 2^63 after theirs
    rng = np.random.default_rng(29)
    for trial in range(60):
        n = int(rng.integers(2, 40000)) if trial % 3 == 0 else int(rng.integers(2, 3000))
        T, Rp = int(rng.integers(1, 65536)), int(rng.integers(1, 6))
        y = (rng.standard_normal(n) * 10.0 ** rng.uniform(-5, 5)).astype(np.float32)
        if trial % 4 == 0:
            y[:] = y[0]
        _, _, s = O.fix_targets(y, T, Rp)
        Rg = s["range"]
        assert (n * Rg * Rg // 4) >> s["s_gain"] < 2 ** 62
        assert (T * Rp * n * (Rg + 1) ** 2) >> s["s_perm"] < 2 ** 63
        assert (n * (Rg + 1) ** 2) >> s["s_kl"] < 2 ** 63


def test_split_search_is_the_squared_error_definition():
    rng = np.random.default_rng(21)
    for trial in range(300):
        n, p, B = int(rng.integers(2, 10)), int(rng.integers(1, 4)), int(rng.integers(2, 7))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        y = exact_targets(rng, n, ties=trial % 5 == 0)
        w = rng.integers(1, 4, n).astype(np.uint32)
        rows = np.arange(n, dtype=np.uint32)
        feats = rng.permutation(p)[: int(rng.integers(1, p + 1))].astype(np.int32)
        yfix, e, sh = O.fix_targets(y)
        got = O.best_split_reg(bins, yfix, w, rows, feats, B, sh["s_gain"])
        want = brute_best_reg(bins, y, w, rows, feats, B)
        if want is None:
            assert got["found"] == 0
            continue
        assert got["found"] == 1
        assert (got["q"], got["b"], got["wl"], got["wr"]) == \
            (want["q"], want["b"], want["wl"], want["wr"])
        # the decrease in fixed-point units, floored after the gain shift
        d_fix = want["d"] * Fraction(2) ** (2 * (38 - e) - sh["s_gain"])
        assert got["gain_fix"] == d_fix.numerator // d_fix.denominator
        # the children's weighted target sums are those of the exact targets
        scale = Fraction(2) ** (38 - e)
        left = [i for i in range(n) if bins[feats[got["q"]]][i] <= got["b"]]
        assert Fraction(got["tl"]) == scale * sum(int(w[i]) * exact(y[i]) for i in left)


def test_root_split_matches_scikit_learn_regression_tree():
    # bootstrap off (unit weights) and every feature drawn: the root split is
    # greedy CART on the bins.  Where the best split is unique by a clear
    # margin, scikit-learn's squared-error tree (float64 sums) picks the same
    # feature and threshold b <-> b + 0.5 and the same left count.
    tree = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(30)
    checked = 0
    for trial in range(80):
        n, p, B = int(rng.integers(20, 200)), int(rng.integers(2, 6)), int(rng.integers(3, 12))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        y = (2.0 * (bins[0] > B // 2) + rng.standard_normal(n) * 0.7).astype(np.float32)
        w = np.ones(n, np.uint32)
        feats = np.arange(p, dtype=np.int32)
        yfix, e, sh = O.fix_targets(y)
        got = O.best_split_reg(bins, yfix, w, np.arange(n, dtype=np.uint32), feats, B,
                               sh["s_gain"])
        if not got["found"]:
            continue
        # margin: the second best (f, b) must be clearly worse
        scores = []
        for f in range(p):
            for b in range(B - 1):
                m = bins[f] <= b
                if m.all() or not m.any():
                    continue
                yl, yr = y[m].astype(np.float64), y[~m].astype(np.float64)
                scores.append((yl.sum() ** 2 / len(yl) + yr.sum() ** 2 / len(yr), f, b))
        scores.sort(reverse=True)
        best_part = bins[scores[0][1]] <= scores[0][2]
        second = [s for s in scores if not np.array_equal(bins[s[1]] <= s[2], best_part)]
        if second and scores[0][0] - second[0][0] < 1e-6 * abs(scores[0][0]):
            continue
        dt = tree.DecisionTreeRegressor(max_depth=1, random_state=0)
        dt.fit(bins.T.astype(np.float64), y.astype(np.float64))
        f_sk, thr_sk = int(dt.tree_.feature[0]), float(dt.tree_.threshold[0])
        part_sk = bins[f_sk] <= thr_sk
        part_or = bins[feats[got["q"]]] <= got["b"]
        assert np.array_equal(part_sk, part_or)
        assert got["wl"] == int(part_or.sum())
        checked += 1
    assert checked >= 40


def test_planted_regression_features_recovered():
    X, y = _problem(24)
    r = O.boruta_fit_reg(X, y, 40, 8, max_iter=30, seed=5, n_bins=64)
    assert list(r["decision"][:3]) == [1, 1, 1]
    assert (r["decision"][3:] <= 0).all()
    assert (r["decision"][3:] == -1).sum() >= 6
    assert list(r["rank"][:3]) == [1, 1, 1]


def test_planted_regression_beyond_65536_rows():
    # the fixed-point sums have no row cap short of the general n <= 2^24
    rng = np.random.default_rng(31)
    n, p = 70000, 5
    X = rng.random((n, p)).astype(np.float32)
    y = (6 * X[:, 0] + 2 * (X[:, 1] > 0.5) + 0.5 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, 8, 4, max_iter=12, seed=3, n_bins=32, trace=True)
    assert list(r["decision"][:2]) == [1, 1]
    tr = r["traces"][0]
    roots = tr["nodes"][tr["nodes"][:, 1] == 1]
    assert (roots[:, 4] == n).all()  # the bootstrap weights of a tree sum to n


def test_regression_arguments_checked():
    X = np.zeros((10, 3), np.float32)
    with pytest.raises(ValueError):
        O.boruta_fit_reg(X, np.arange(10, dtype=np.float32), 2, 2, importance_mode=3)
    y = np.arange(10, dtype=np.float32)
    y[3] = np.inf
    with pytest.raises(ValueError):
        O.boruta_fit_reg(X, y, 2, 2)


def _columns(tr, bins, seed, n):
    p_cur = tr["p_cur"]

    def column(fw):
        src = tr["col_src"][fw]
        if fw < p_cur:
            return bins[src].astype(np.int64)
        s = fw - p_cur
        return np.array([bins[src][O.keyed_perm(seed, 3, 1, s, 0, 0, n, i)] for i in range(n)],
                        np.int64)
    return column


def _stump_leaves(tr, tau, col, b, w, yfix):
    """floor(T / W) of the in-bag rows on each side of a root split."""
    v = {}
    for side in (True, False):
        m_in = (w > 0) & ((col <= b) == side)
        T, W = int((w[m_in] * yfix[m_in]).sum()), int(w[m_in].sum())
        v[side] = T // W  # Python's // floors toward minus infinity
    return v


def test_permutation_importance_of_stumps_recomputed_in_python():
    # Permut for regression on depth-1 trees, recomputed here from the
    # definition: the leaf predictions floor(T / W) of the in-bag rows on each
    # side of the root split, squared errors shifted by s_perm, and the OOB
    # rows' error increase when the root column's bins are moved by the keyed
    # permutation of the OOB set (shadow columns rebuilt by their own keyed
    # row permutation)
    rng = np.random.default_rng(25)
    n, p, B, T, R, seed = 400, 6, 16, 7, 2, 9
    X = rng.random((n, p)).astype(np.float32)
    y = (3 * X[:, 0] + np.sin(5 * X[:, 1]) + 0.3 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, T, 1, importance_mode=1, max_iter=1, seed=seed, n_bins=B,
                         n_perm=R, trace=True)
    tr = r["traces"][0]
    bins, _, _ = O.bin_matrix(X, B)
    yfix, e, sh = O.fix_targets(y, T, R)
    column = _columns(tr, bins, seed, n)
    want = np.zeros(tr["p_w"], object)
    oob_total = 0
    for tau in range(T):
        w = O.bootstrap(seed, 1, tau, n).astype(np.int64)
        root = tr["nodes"][(tr["nodes"][:, 0] == tau) & (tr["nodes"][:, 1] == 1)][0]
        f, b = int(root[2]), int(root[3])
        oob = np.flatnonzero(w == 0)
        oob_total += len(oob)
        if f < 0:
            continue
        col = column(f)
        v = _stump_leaves(tr, tau, col, b, w, yfix)
        m = len(oob)
        for rep in range(R):
            for j in range(m):
                src = O.keyed_perm(seed, 4, 1, tau, f, rep << 16, m, j)
                e1 = v[bool(col[oob[src]] <= b)] - int(yfix[oob[j]])
                e0 = v[bool(col[oob[j]] <= b)] - int(yfix[oob[j]])
                want[f] += (e1 * e1 >> sh["s_perm"]) - (e0 * e0 >> sh["s_perm"])
    assert [int(v) for v in tr["imp_int"]] == [int(v) for v in want]
    assert want[0] > 0
    # reported in squared target units: drop / (R * OOB rows) * 2^(s_perm - 2 (38 - e))
    got = r["imp_history"][0, 0]
    assert got == np.ldexp(float(want[0]) / (R * oob_total), sh["s_perm"] - 2 * (38 - e))


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


def test_leaf_predictions_and_tree_table():
    # every leaf of a traced tree predicts floor(T / W) of its in-bag rows,
    # its weighted count is W, and a split's children partition its rows
    X, y = _problem(32, n=300, p=4)
    T, seed = 3, 11
    r = O.boruta_fit_reg(X, y, T, 3, max_iter=1, seed=seed, n_bins=16, trace=True)
    tr = r["traces"][0]
    bins, _, _ = O.bin_matrix(X, 16)
    yfix, _, _ = O.fix_targets(y)
    column = _columns(tr, bins, seed, X.shape[0])
    for tau in range(T):
        w = O.bootstrap(seed, 1, tau, X.shape[0]).astype(np.int64)
        nodes = {int(nd[1]): nd for nd in tr["nodes"][tr["nodes"][:, 0] == tau]}

        def rows_of(h):
            m = w > 0
            path = []
            while h > 1:
                path.append(h)
                h //= 2
            h = 1
            for c in reversed(path):
                f, b = int(nodes[h][2]), int(nodes[h][3])
                m = m & ((column(f) <= b) == (c == 2 * h))
                h = c
            return m

        for h, nd in nodes.items():
            m = rows_of(h)
            W, Tt = int(w[m].sum()), int((w[m] * yfix[m]).sum())
            assert int(nd[4]) == W
            if nd[2] < 0:
                assert int(nd[3]) == Tt // W


def test_divergence_importance_of_stumps_recomputed_in_python():
    # Algorithm 3 for regression on depth-1 trees, recomputed here: the shared
    # row permutation of the iteration, per row the change D of the summed
    # leaf predictions floor(T / W) when the column is permuted, and the sum
    # over rows of floor(D^2 / n_trees^2) shifted by s_kl
    rng = np.random.default_rng(28)
    n, p, B, T, seed = 300, 5, 16, 6, 4
    X = rng.random((n, p)).astype(np.float32)
    y = (3 * X[:, 0] + np.sin(5 * X[:, 1]) + 0.3 * rng.standard_normal(n)).astype(np.float32)
    r = O.boruta_fit_reg(X, y, T, 1, importance_mode=2, max_iter=1, seed=seed, n_bins=B,
                         trace=True)
    tr = r["traces"][0]
    bins, _, _ = O.bin_matrix(X, B)
    yfix, e, sh = O.fix_targets(y, T, 1)
    column = _columns(tr, bins, seed, n)
    pi = np.array([O.keyed_perm(seed, 5, 1, 0, 0, 0, n, i) for i in range(n)])
    stumps = []
    for tau in range(T):
        w = O.bootstrap(seed, 1, tau, n).astype(np.int64)
        root = tr["nodes"][(tr["nodes"][:, 0] == tau) & (tr["nodes"][:, 1] == 1)][0]
        f, b = int(root[2]), int(root[3])
        if f < 0:
            continue
        col = column(f)
        stumps.append((f, b, col, _stump_leaves(tr, tau, col, b, w, yfix)))
    want = [0] * tr["p_w"]
    for f in range(tr["p_w"]):
        for row in range(n):
            d = 0
            for (g, b, col, v) in stumps:
                if g == f:
                    d += v[bool(col[pi[row]] <= b)] - v[bool(col[row] <= b)]
            want[f] += (d * d // (T * T)) >> sh["s_kl"]
    assert [int(v) for v in tr["imp_int"]] == want
    assert want[0] > 0
    got = r["imp_history"][0, 0]
    assert got == np.ldexp(float(want[0]) / n, sh["s_kl"] - 2 * (38 - e))
