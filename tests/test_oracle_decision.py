"""Pins of the oracle's Bonferroni binomial decision: exact rational tails
(math.comb), scipy's binomial survival/cumulative functions, and the closed
form of the earliest possible decision."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def exact(h, t, p, alpha):
    a = Fraction(alpha)
    up = Fraction(sum(math.comb(t, k) for k in range(h, t + 1)), 2**t)
    lo = Fraction(sum(math.comb(t, k) for k in range(0, h + 1)), 2**t)
    if p * up < a:
        return 1
    if p * lo < a:
        return -1
    return 0


def test_exhaustive_small_t():
    for t in range(1, 41):
        for h in range(t + 1):
            for p in (1, 3, 20, 500):
                for alpha in (0.05, 0.01, 0.3):
                    assert O.binom_decide(h, t, p, alpha) == exact(h, t, p, alpha)


def test_random_large_t_exact_and_scipy():
    rng = np.random.default_rng(0)
    for _ in range(400):
        t = int(rng.integers(1, 1001))
        h = int(rng.integers(0, t + 1))
        if rng.random() < 0.5:  # concentrate near the decision boundaries
            h = int(np.clip(round(t / 2 + rng.normal(0, 2) * math.sqrt(t)), 0, t))
        p = int(rng.integers(1, 30000))
        alpha = float(rng.uniform(1e-4, 0.49))
        got = O.binom_decide(h, t, p, alpha)
        assert got == exact(h, t, p, alpha)
        up = p * stats.binom.sf(h - 1, t, 0.5)
        lo = p * stats.binom.cdf(h, t, 0.5)
        if abs(up - alpha) > 1e-9 * alpha and abs(lo - alpha) > 1e-9 * alpha:
            want = 1 if up < alpha else (-1 if lo < alpha else 0)
            assert got == want


@pytest.mark.parametrize("p,t_star", [(20, 9), (500, 14), (20000, 19), (50, 10), (2000, 16)])
def test_earliest_decision_closed_form(p, t_star):
    alpha = 0.05
    assert t_star == min(t for t in range(1, 100) if 2**t > p / alpha)
    for t in range(1, t_star):
        assert O.binom_decide(t, t, p, alpha) == 0
        assert O.binom_decide(0, t, p, alpha) == 0
    assert O.binom_decide(t_star, t_star, p, alpha) == 1
    assert O.binom_decide(0, t_star, p, alpha) == -1


def test_monotone_thresholds():
    for t in (15, 60, 300):
        d = [O.binom_decide(h, t, 100, 0.05) for h in range(t + 1)]
        # -1 ... -1, 0 ... 0, 1 ... 1
        assert d == sorted(d)


def test_final_ranking_of_algorithm1():
    # hand-computed: features 0 and 3 confirmed, 4 undecided, 1, 2, 5 rejected
    # with mean history (over their finite entries) 0.2, 0.35, 0.35 -> ranks
    # 5, 3, 3 (equal means share the smaller rank)
    nan = np.nan
    hist = np.array([[0.5, 0.1, 0.4, 0.6, 0.2, 0.3],
                     [0.6, 0.3, 0.3, 0.7, 0.1, 0.4],
                     [0.7, nan, nan, 0.8, 0.3, nan],
                     [9.0, 9.0, 9.0, 9.0, 9.0, 9.0]])  # past n_iter: ignored
    dec = np.array([1, -1, -1, 1, 0, -1], np.int8)
    r = O.rank(dec, hist, 3)
    assert list(r) == [1, 5, 3, 1, 2, 3]


def test_final_ranking_properties_on_a_run():
    from paper_2605_09950_amd import synth
    c = synth.config(0)
    pr = c["params"]
    out = O.boruta_fit(c["X"], c["y"], 2, pr["n_trees"], pr["max_depth"], max_iter=pr["max_iter"],
                       seed=c["seed"], n_bins=pr["n_bins"])
    r, d, h = out["rank"], out["decision"], out["imp_history"][: out["n_iter"]]
    assert np.all(r[d == 1] == 1) and np.all(r[d == 0] == 2) and np.all(r[d == -1] >= 3)
    rej = np.flatnonzero(d == -1)
    m = {j: np.nanmean(h[:, j]) for j in rej}
    for a in rej:
        for b in rej:
            if m[a] > m[b] + 1e-12:
                assert r[a] < r[b]
    assert r[rej].min() == 3


def test_seed_median_hand_computed_and_library_median():
    import statistics
    nan = np.nan
    # two features, three runs of up to three iterations
    runs = [dict(decision=np.array([1, -1], np.int8), n_iter=3,
                 imp_history=np.array([[0.5, 0.1], [0.7, nan], [0.6, nan]])),
            dict(decision=np.array([1, 0], np.int8), n_iter=2,
                 imp_history=np.array([[0.2, 0.3], [0.4, 0.1], [9.0, 9.0]])),
            dict(decision=np.array([0, -1], np.int8), n_iter=1,
                 imp_history=np.array([[0.9, 0.05], [9.0, 9.0], [9.0, 9.0]]))]
    med, dec = O.seed_median(runs)
    # feature 0: means 0.6, 0.3, 0.9 -> 0.6; feature 1: 0.1, 0.2, 0.05 -> 0.1
    assert med[0] == (0.5 + 0.7 + 0.6) / 3 and med[1] == 0.1
    assert list(dec) == [1, -1]
    # even count: mean of the middle pair; decisions: lower median
    med2, dec2 = O.seed_median(runs[:2])
    assert med2[0] == ((0.5 + 0.7 + 0.6) / 3 + (0.2 + 0.4) / 2) / 2
    assert list(dec2) == [1, -1]
    rng = np.random.default_rng(3)
    runs = []
    for r in range(7):
        h = rng.random((5, 4))
        n_it = int(rng.integers(1, 6))
        runs.append(dict(decision=rng.integers(-1, 2, 4).astype(np.int8), n_iter=n_it,
                         imp_history=h))
    med, dec = O.seed_median(runs)
    for j in range(4):
        means = [sum(float(r["imp_history"][t][j]) for t in range(r["n_iter"])) / r["n_iter"]
                 for r in runs]
        assert med[j] == statistics.median(means)
        assert dec[j] == statistics.median_low([int(r["decision"][j]) for r in runs])


def test_shadow_threshold_is_numpys_inverted_cdf_percentile():
    # nearest-rank percentile = numpy's "inverted_cdf" method; 100 = maximum
    rng = np.random.default_rng(8)
    for m in (1, 2, 5, 7, 40, 333):
        for _ in range(3):
            a = rng.integers(-50, 50, m) * int(rng.integers(1, 2**40))
            assert O.shadow_threshold(a, 100) == a.max()
            for q in (1, 10, 25, 33, 50, 67, 75, 90, 99):
                want = np.percentile(a, q, method="inverted_cdf")
                assert O.shadow_threshold(a, q) == int(want)
    # hand-computed: sorted [1, 3, 5, 9]; ranks ceil(q * 4 / 100)
    assert [O.shadow_threshold([5, 1, 9, 3], q) for q in (1, 25, 26, 50, 51, 75, 76, 100)] == \
        [1, 1, 3, 3, 5, 5, 9, 9]


def test_rough_fix_hand_computed_and_library_median():
    nan = np.nan
    dec = np.array([0, 1, 0, -1, 0], np.int8)
    hist = np.array([[0.30, 0.9, 0.10, 0.5, 0.20],
                     [0.10, 0.8, 0.05, nan, 0.25],
                     [0.40, 0.7, 0.20, nan, 0.15],
                     [9.00, 9.0, 9.00, 9.0, 9.00]])
    smax = np.array([0.2, 0.2, 0.25, 7.0])
    # three iterations: shadow median 0.2; tentative medians 0.30, 0.10, 0.20
    out = O.rough_fix(dec, hist, smax, 3)
    assert list(out) == [1, 1, -1, -1, -1]  # equal to the shadow median is not above it
    assert list(O.rough_fix(dec, hist, smax, 0)) == list(dec)
    # two iterations (even count): shadow median 0.2; medians 0.2, 0.075, 0.225
    assert list(O.rough_fix(dec, hist, smax, 2)) == [-1, 1, -1, -1, 1]
    rng = np.random.default_rng(12)
    for _ in range(20):
        p, t = int(rng.integers(1, 9)), int(rng.integers(1, 8))
        dec = rng.integers(-1, 2, p).astype(np.int8)
        hist = rng.random((t + 2, p))
        smax = rng.random(t + 2)
        out = O.rough_fix(dec, hist, smax, t)
        ms = np.median(smax[:t])
        for j in range(p):
            want = dec[j] if dec[j] != 0 else (1 if np.median(hist[:t, j]) > ms else -1)
            assert out[j] == want


def test_percentile_and_rough_fix_on_runs():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 10)).astype(np.float32)
    y = (X[:, 0] + 0.5 * X[:, 1] + 0.7 * rng.standard_normal(300) > 0).astype(np.int32)
    kw = dict(n_bins=32, seed=3)
    base = O.boruta_fit(X, y, 2, 10, 6, max_iter=12, **kw)
    same = O.boruta_fit(X, y, 2, 10, 6, max_iter=12, perc=100, **kw)
    assert np.array_equal(base["decision"], same["decision"])
    assert np.array_equal(base["imp_history"], same["imp_history"], equal_nan=True)
    # the first iteration's forest does not depend on the threshold: a lower
    # percentile gives every feature at least its hits against the maximum
    h100 = O.boruta_fit(X, y, 2, 10, 6, max_iter=1, **kw)["hits"]
    for q in (90, 50, 10):
        hq = O.boruta_fit(X, y, 2, 10, 6, max_iter=1, perc=q, **kw)["hits"]
        assert (hq >= h100).all()
    # the rough fix only post-processes the finished run
    fixed = O.boruta_fit(X, y, 2, 10, 6, max_iter=12, rough_fix=True, **kw)
    assert np.array_equal(fixed["imp_history"], base["imp_history"], equal_nan=True)
    want = O.rough_fix(base["decision"], base["imp_history"], base["shadow_max"], base["n_iter"])
    assert np.array_equal(fixed["decision"], want)
    assert (base["decision"] == 0).any() and not (fixed["decision"] == 0).any()
    assert not (fixed["rank"] == 2).any()
