"""Pins of the oracle's importance scores.

TreeImp is checked against a literal double-precision transcription of
Algorithm 2 (per-node decrease x count summed per feature, per-tree
normalisation, mean over trees, renormalisation) computed from the traced
trees by routing the rows again; Permut against a direct recount of the
out-of-bag accuracy drop and against its own naive full re-traversal.  The
prediction-divergence importance of Algorithm 3 (mode 2) is checked through
its parts: the fixed-point log2 against 60-digit decimal logarithms, the
fixed-point KL against scipy's entropy, the whole score against a recount
from leaf class counts routed afresh, and a pure stump's closed form."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.oracle_helpers import (gini_decrease_fraction, leaf_of, route_counts, tree_dict,
                                  widened)


def _problem(seed, n=160, p=6, K=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(np.float32)
    y = ((X[:, 0] > 0).astype(int) + (X[:, 1] > 0.5).astype(int) + rng.integers(0, 2, n)) % K
    return X, y.astype(np.int32)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_treeimp_matches_literal_algorithm2(seed):
    X, y = _problem(seed)
    K, T, D, B = 3, 7, 5, 32
    state = np.zeros(X.shape[1], np.int8)
    state[4] = -1  # a rejected column must be left out of the widened matrix
    out = O.boruta_step(X, y, K, T, D, t=2, state=state, hits=np.zeros(X.shape[1], np.int32),
                        importance_mode=0, seed=seed, n_bins=B)
    tr = out["trace"]
    W, active, n_sha = widened(X, state, 2, seed, B)
    assert list(tr["col_src"][: len(active)]) == active and tr["n_sha"] == n_sha
    p_w = W.shape[0]
    imp_trees = np.zeros((T, p_w))
    for tree in range(T):
        w = O.bootstrap(seed, 2, tree, X.shape[0])
        td = tree_dict(tr["nodes"], tree)
        cnt = route_counts(td, W, np.flatnonzero(w), w, y, K)
        fg = np.zeros(p_w)
        for h, r in td.items():
            assert int(r[4]) == int(cnt[h].sum())
            if int(r[2]) < 0:
                continue
            cp, cl, cr = cnt[h], cnt[2 * h], cnt[2 * h + 1]
            exact = gini_decrease_fraction(cp, cl, cr)
            assert int(r[5]) == (exact * 2**32).numerator // (exact * 2**32).denominator
            # literal double-precision Algorithm 2: gain x instance_count
            def gini(c):
                return 1.0 - float(((c / c.sum()) ** 2).sum())
            gain = gini(cp) - cl.sum() / cp.sum() * gini(cl) - cr.sum() / cp.sum() * gini(cr)
            fg[int(r[2])] += gain * cp.sum()
        if fg.sum() > 0:
            imp_trees[tree] = fg / fg.sum()
    imp = imp_trees.mean(axis=0)
    ref = imp / imp.sum()
    got = tr["imp_int"] / tr["imp_int"].sum()
    big = ref >= 1e-7
    assert np.all(np.abs(got[big] - ref[big]) <= 1e-6 * ref[big])
    assert np.all(np.abs(got[~big] - ref[~big]) <= 1e-13)
    # reported row: active originals carry I/sum(I), rejected ones NaN
    assert np.isnan(out["imp_row"][4])
    for c, j in enumerate(active):
        assert out["imp_row"][j] == tr["imp_int"][c] / tr["imp_int"].sum()


def test_single_split_tree_gives_unit_importance():
    # column 0 separates the classes exactly; depth 1 -> one split per tree
    n = 200
    X = np.zeros((n, 3), np.float32)
    X[:, 0] = np.arange(n)
    X[:, 1:] = np.random.default_rng(0).standard_normal((n, 2))
    y = (X[:, 0] >= n / 2).astype(np.int32)
    out = O.boruta_step(X, y, 2, 4, 1, t=1, state=np.zeros(3, np.int8),
                        hits=np.zeros(3, np.int32), mtry=100, seed=5, n_bins=64)
    tr = out["trace"]
    assert tr["imp_int"][0] == 4 * 2**44 and tr["imp_int"][1:].sum() == 0
    assert out["imp_row"][0] == 1.0


@pytest.mark.parametrize("seed", [4, 5])
def test_permut_naive_equals_path_restricted(seed):
    X, y = _problem(seed, n=120, p=5)
    kw = dict(importance_mode=1, seed=seed, n_bins=16, n_perm=3)
    st = np.zeros(5, np.int8)
    a = O.boruta_step(X, y, 3, 6, 4, t=1, state=st, hits=np.zeros(5, np.int32), **kw)
    b = O.boruta_step(X, y, 3, 6, 4, t=1, state=st, hits=np.zeros(5, np.int32),
                      permut_naive=True, **kw)
    assert np.array_equal(a["trace"]["imp_int"], b["trace"]["imp_int"])
    assert np.array_equal(a["hits"], b["hits"])


def test_permut_matches_direct_recount():
    seed, R, t = 6, 2, 3
    X, y = _problem(seed, n=90, p=4)
    state = np.zeros(4, np.int8)
    out = O.boruta_step(X, y, 3, 5, 4, t=t, state=state, hits=np.zeros(4, np.int32),
                        importance_mode=1, seed=seed, n_bins=16, n_perm=R)
    tr = out["trace"]
    W, active, n_sha = widened(X, state, t, seed, 16)
    p_w = W.shape[0]
    drop = np.zeros(p_w, np.int64)
    oob_total = 0
    for tree in range(5):
        w = O.bootstrap(seed, t, tree, X.shape[0])
        oob = np.flatnonzero(w == 0)
        m = len(oob)
        oob_total += m
        td = tree_dict(tr["nodes"], tree)
        base = [int(td[leaf_of(td, W, r)][3]) == y[r] for r in oob]
        assert sum(base) == tr["tree_stats"][tree][3]
        for f in range(p_w):
            for r in range(R):
                for j in range(m):
                    src = O.keyed_perm(seed, O.STREAM_OOBPERM, t, tree, f, r << 16, m, j)
                    pred = int(td[leaf_of(td, W, oob[j], f, int(W[f][oob[src]]))][3])
                    drop[f] += int(base[j]) - int(pred == y[oob[j]])
    assert np.array_equal(drop, tr["imp_int"])
    used = {int(r[2]) for r in tr["nodes"] if r[2] >= 0}
    for f in range(p_w):
        if f not in used:
            assert tr["imp_int"][f] == 0
    for c, j in enumerate(active):
        assert out["imp_row"][j] == drop[c] / (R * oob_total)


def test_permut_identity_when_oob_tiny():
    # n = 2: every tree has at most one OOB row, so every permutation is the identity
    X = np.array([[0.0, 1.0], [1.0, 0.0]], np.float32)
    y = np.array([0, 1], np.int32)
    out = O.boruta_step(X, y, 2, 8, 2, t=1, state=np.zeros(2, np.int8),
                        hits=np.zeros(2, np.int32), importance_mode=1, seed=1, n_bins=4)
    assert np.all(out["trace"]["imp_int"] == 0)


# ---------------------------------------------------------------------------
# Importance mode 2: Algorithm 3 (shared row permutation, forest class
# probabilities on the full training matrix, KL divergence in bits with 32
# fractional bits, summed over rows).

def _log2_exact_units(x):
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    return Decimal(x).ln() / Decimal(2).ln() * Decimal(2**32)


def test_log2_fix32_digit_method():
    # exact at powers of two; otherwise at most two units below 2^32 log2 x
    # (each of the 32 squarings truncates the 62-bit mantissa)
    for e in range(0, 62):
        assert O.log2_fix32(2**e) == e << 32
    rng = np.random.default_rng(9)
    xs = [3, 5, 7, 10, 1000, 2**32 - 1, 2**32 + 1, 3 * 2**40 + 17]
    xs += [int(v) for v in rng.integers(1, 2**48, 300)]
    for x in xs:
        ref = _log2_exact_units(x)
        got = O.log2_fix32(x)
        assert ref - 2 <= got <= ref, (x, got, ref)


def test_kl_fix32_matches_library_divergence():
    from scipy.stats import entropy
    rng = np.random.default_rng(10)
    for K in (2, 3, 4, 7):
        for _ in range(60):
            S = rng.integers(0, 2**36, K).astype(np.uint64)
            S[rng.integers(0, K)] = 0 if K > 2 and rng.random() < 0.3 else S[0]
            if S.sum() == 0:
                S[0] = 1
            Sq = rng.integers(0, 2**36, K).astype(np.uint64)
            if rng.random() < 0.2:
                Sq[rng.integers(0, K)] = 0
            if rng.random() < 0.2:
                Sq = S.copy()  # identical predictions: exactly zero
            got = O.kl_fix32(S, Sq)
            q = np.where((Sq == 0) & (S > 0), 1, Sq).astype(np.float64)
            ref = entropy(S.astype(np.float64), q, base=2)  # normalises both
            assert abs(got / 2**32 - ref) <= 4 * 2**-32 * max(1.0, ref), (S, Sq, got, ref)
            if np.array_equal(S, Sq):
                assert got == 0
    # a class the permuted prediction misses gets one unit: p = (1, 0), q = (0, 1)
    assert abs(O.kl_fix32([2**32, 0], [0, 2**32]) / 2**32 - 32.0) < 1e-9


def _forest_probs(tr, W, y, K, seed, t, T, n):
    """Per tree: leaf class counts of the in-bag rows, routed afresh."""
    out = []
    for tree in range(T):
        w = O.bootstrap(seed, t, tree, n)
        td = tree_dict(tr["nodes"], tree)
        cnt = route_counts(td, W, np.flatnonzero(w), w, y, K)
        out.append((td, cnt))
    return out


def _predict_fix(forest, W, row, K, sub_f=-1, sub_b=0):
    S = np.zeros(K, dtype=np.uint64)
    for td, cnt in forest:
        c = cnt[leaf_of(td, W, row, sub_f, sub_b)]
        N = int(c.sum())
        S += np.array([(int(v) << 32) // N for v in c], dtype=np.uint64)
    return S


@pytest.mark.parametrize("seed", [11, 12])
def test_kl_importance_matches_direct_recount(seed):
    X, y = _problem(seed, n=80, p=4)
    K, T, D, B, t = 3, 4, 4, 16, 2
    state = np.zeros(4, np.int8)
    out = O.boruta_step(X, y, K, T, D, t=t, state=state, hits=np.zeros(4, np.int32),
                        importance_mode=2, seed=seed, n_bins=B)
    tr = out["trace"]
    W, active, n_sha = widened(X, state, t, seed, B)
    n, p_w = X.shape[0], W.shape[0]
    forest = _forest_probs(tr, W, y, K, seed, t, T, n)
    pi = [O.keyed_perm(seed, O.STREAM_FLUSH, t, 0, 0, 0, n, r) for r in range(n)]
    assert sorted(pi) == list(range(n))
    base = [_predict_fix(forest, W, r, K) for r in range(n)]
    imp = np.zeros(p_w, np.int64)
    imp_float = np.zeros(p_w)
    from scipy.stats import entropy
    for f in range(p_w):
        for r in range(n):
            q = _predict_fix(forest, W, r, K, f, int(W[f][pi[r]]))
            imp[f] += O.kl_fix32(base[r], q)
            qq = np.where((q == 0) & (base[r] > 0), 1, q).astype(float)
            imp_float[f] += entropy(base[r].astype(float), qq, base=2)
    assert np.array_equal(imp, tr["imp_int"])
    assert np.all(np.abs(imp / 2**32 - imp_float) <= n * 4 * 2**-32 * np.maximum(1, imp_float))
    used = {int(r[2]) for r in tr["nodes"] if r[2] >= 0}
    for f in range(p_w):
        if f not in used:
            assert tr["imp_int"][f] == 0
    for c, j in enumerate(active):
        assert out["imp_row"][j] == imp[c] / (n * 2**32)
    best = max(imp[len(active):])
    assert np.array_equal(out["hits"], np.array([1 if imp[c] > best else 0
                                                  for c in range(len(active))], np.int32))


def test_kl_importance_of_a_pure_stump():
    # one tree of depth 1 splitting column 0, whose bins separate the two
    # classes: every leaf is pure, so a row whose permuted bin falls on the
    # other side of the threshold moves from p = (1, 0) to q = (0, 1) and adds
    # KL = 32 + log2(1 + 2^-32) bits (the missing class gets one unit); rows
    # that stay add nothing.  Other columns are never tested.
    n = 64
    X = np.zeros((n, 2), np.float32)
    X[:, 0] = np.arange(n)
    X[:, 1] = np.random.default_rng(1).standard_normal(n)
    y = (X[:, 0] >= n / 2).astype(np.int32)
    seed, t = 3, 1
    out = O.boruta_step(X, y, 2, 1, 1, t=t, state=np.zeros(2, np.int8),
                        hits=np.zeros(2, np.int32), mtry=100, importance_mode=2, seed=seed,
                        n_bins=64)
    tr = out["trace"]
    root = [r for r in tr["nodes"] if r[1] == 1][0]
    assert root[2] == 0
    bins, _, _ = O.bin_matrix(X, 64)
    thr = int(root[3])
    side = bins[0] <= thr
    pi = [O.keyed_perm(seed, O.STREAM_FLUSH, t, 0, 0, 0, n, r) for r in range(n)]
    moved = sum(1 for r in range(n) if side[r] != side[pi[r]])
    assert moved > 0
    per_row = O.kl_fix32([2**32, 0], [0, 2**32])
    assert per_row == (32 << 32) + O.log2_fix32(2**32 + 1) - (32 << 32)
    assert tr["imp_int"][0] == moved * per_row
    assert np.all(tr["imp_int"][1:] == 0)
