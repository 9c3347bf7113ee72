"""Pins of the oracle's split search and tree growth: exhaustive brute force
with exact rationals, and scikit-learn's CART on the special case without
bootstrap and with every feature drawn."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def brute_best(bins, y, w, rows, feats, K, B):
    """Every (draw position, threshold) scored with exact fractions; the first
    maximum in (position, threshold) order wins; split iff strictly better
    than the parent's S/N."""
    counts = [sum(int(w[i]) for i in rows if y[i] == k) for k in range(K)]
    N = sum(counts)
    S = sum(c * c for c in counts)
    best = None
    for q, f in enumerate(feats):
        for b in range(B - 1):
            cl = [sum(int(w[i]) for i in rows if y[i] == k and bins[f][i] <= b) for k in range(K)]
            cr = [counts[k] - cl[k] for k in range(K)]
            nl, nr = sum(cl), sum(cr)
            if nl == 0 or nr == 0:
                continue
            Q = Fraction(sum(c * c for c in cl), nl) + Fraction(sum(c * c for c in cr), nr)
            if best is None or Q > best[0]:
                best = (Q, q, b, nl, nr)
    if best is None or not best[0] > Fraction(S, N):
        return None
    gain = best[0] - Fraction(S, N)
    return dict(q=best[1], b=best[2], nl=best[3], nr=best[4],
                gain_fix=(gain * 2**32).numerator // (gain * 2**32).denominator)


def test_all_labelings_tiny():
    rng = np.random.default_rng(0)
    for trial in range(40):
        n, p, B = int(rng.integers(2, 7)), int(rng.integers(1, 4)), int(rng.integers(2, 5))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        w = rng.integers(1, 3, n).astype(np.uint32)
        rows = np.arange(n, dtype=np.uint32)
        feats = rng.permutation(p).astype(np.int32)
        for lab in itertools.product(range(2), repeat=n):
            y = np.array(lab, np.int32)
            got = O.best_split(bins, y, w, rows, feats, 2, B)
            want = brute_best(bins, y, w, rows, feats, 2, B)
            if want is None:
                assert got["found"] == 0
            else:
                assert got["found"] == 1
                assert (got["q"], got["b"], got["nl"], got["nr"], got["gain_fix"]) == \
                    (want["q"], want["b"], want["nl"], want["nr"], want["gain_fix"])


@pytest.mark.parametrize("K", [3, 4])
def test_random_multiclass(K):
    rng = np.random.default_rng(K)
    for trial in range(150):
        n, p, B = int(rng.integers(2, 12)), int(rng.integers(1, 5)), int(rng.integers(2, 9))
        bins = rng.integers(0, B, size=(p, n)).astype(np.uint8)
        y = rng.integers(0, K, n).astype(np.int32)
        w = rng.integers(0, 4, n).astype(np.uint32)
        rows = np.flatnonzero(w).astype(np.uint32)
        if len(rows) == 0:
            continue
        feats = rng.permutation(p)[: int(rng.integers(1, p + 1))].astype(np.int32)
        got = O.best_split(bins, y, w, rows, feats, K, B)
        want = brute_best(bins, y, w, rows, feats, K, B)
        if want is None:
            assert got["found"] == 0
        else:
            assert got["found"] == 1
            assert (got["q"], got["b"], got["nl"], got["nr"], got["gain_fix"]) == \
                (want["q"], want["b"], want["nl"], want["nr"], want["gain_fix"])


def test_tie_breaks_to_first_draw_then_smallest_threshold():
    # two identical columns: the one drawn first wins; within it, the smallest b
    bins = np.array([[0, 0, 3, 3], [0, 0, 3, 3]], np.uint8)
    y = np.array([0, 0, 1, 1], np.int32)
    w = np.ones(4, np.uint32)
    rows = np.arange(4, dtype=np.uint32)
    got = O.best_split(bins, y, w, rows, np.array([1, 0], np.int32), 2, 4)
    assert got["found"] == 1 and got["q"] == 0 and got["b"] == 0
    got = O.best_split(bins, y, w, rows, np.array([0, 1], np.int32), 2, 4)
    assert got["q"] == 0 and got["b"] == 0
    # pure node: never split
    y1 = np.zeros(4, np.int32)
    assert O.best_split(bins, y1, w, rows, np.array([0], np.int32), 2, 4)["found"] == 0


def frac_tree(bins, y, w, K, B, D, mtry, seed, t, tree):
    """Recursive tree built with exact fractions, feature draws from the
    oracle's keyed bijection (an input here, pinned separately)."""
    p_w, n = bins.shape
    out = []

    def grow(rows, depth, heap):
        counts = [sum(int(w[i]) for i in rows if y[i] == k) for k in range(K)]
        N = sum(counts)
        split = None
        if depth < D:
            feats = [O.keyed_perm(seed, O.STREAM_MTRY, t, tree, heap, 0, p_w, q)
                     for q in range(mtry)]
            split = brute_best(bins, y, w, rows, feats, K, B)
        if split is None:
            out.append((tree, heap, -1, int(np.argmax(counts)), N, 0))
            return
        f = O.keyed_perm(seed, O.STREAM_MTRY, t, tree, heap, 0, p_w, split["q"])
        out.append((tree, heap, f, split["b"], N, split["gain_fix"]))
        grow([i for i in rows if bins[f][i] <= split["b"]], depth + 1, 2 * heap)
        grow([i for i in rows if bins[f][i] > split["b"]], depth + 1, 2 * heap + 1)

    grow([i for i in range(n) if w[i] > 0], 0, 1)
    return sorted(out, key=lambda r: r[1])


def test_tree_matches_fraction_builder():
    rng = np.random.default_rng(42)
    for trial in range(25):
        n, p_w, B, K = int(rng.integers(4, 30)), int(rng.integers(1, 6)), int(rng.integers(2, 7)), \
            int(rng.integers(2, 4))
        bins = rng.integers(0, B, size=(p_w, n)).astype(np.uint8)
        y = rng.integers(0, K, n).astype(np.int32)
        w = O.bootstrap(trial, 1, 0, n)
        D = int(rng.integers(1, 6))
        mtry = int(rng.integers(1, p_w + 1))
        nodes, _ = O.grow_tree(bins, y, w, K, B, D, mtry, seed=trial, t=1, tree=3)
        want = frac_tree(bins, y, w, K, B, D, mtry, trial, 1, 3)
        assert [tuple(int(v) for v in r) for r in nodes] == want


def test_root_matches_sklearn_cart():
    from sklearn.tree import DecisionTreeClassifier
    rng = np.random.default_rng(9)
    checked = 0
    for trial in range(60):
        n, p_w, B, K = 200, 6, 16, int(rng.integers(2, 5))
        bins = rng.integers(0, B, size=(p_w, n)).astype(np.uint8)
        y = ((bins[trial % p_w] > 7).astype(int) + rng.integers(0, K, n)) % K
        y = y.astype(np.int32)
        w = np.ones(n, np.uint32)
        feats = np.arange(p_w, dtype=np.int32)
        got = O.best_split(bins, y, w, np.arange(n, dtype=np.uint32), feats, K, B)
        # is the best split unique? (second best strictly worse)
        X = bins.T.astype(np.float64)
        clf = DecisionTreeClassifier(criterion="gini", max_depth=1, max_features=None,
                                     random_state=0).fit(X, y)
        if not got["found"]:
            continue
        f = int(feats[got["q"]])
        # compare partitions, not thresholds (sklearn uses midpoints)
        sk_f = clf.tree_.feature[0]
        sk_left = X[:, sk_f] <= clf.tree_.threshold[0]
        ours_left = bins[f] <= got["b"]
        if sk_f == f:
            assert np.array_equal(sk_left, ours_left)
            checked += 1
        else:
            # only an exact tie may differ: both partitions score the same
            def score(mask):
                def s(m):
                    c = np.bincount(y[m], minlength=K)
                    return Fraction(int((c * c).sum()), int(c.sum()))
                return s(mask) + s(~mask)
            assert score(sk_left) == score(ours_left)
    assert checked > 40
