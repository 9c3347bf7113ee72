"""Whole-run checks of the oracle's Boruta loop (Algorithm 1): planted
recovery, determinism, resumability from (state, hits), the history's NaN
pattern, final decisions, shadow doubling and argument validation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_09950_amd import synth


@pytest.fixture(scope="module")
def run0():
    c = synth.config(0)
    pr = c["params"]
    r = O.boruta_fit(c["X"], c["y"], c["n_classes"], pr["n_trees"], pr["max_depth"],
                     max_iter=pr["max_iter"], seed=c["seed"], n_bins=pr["n_bins"], trace=True)
    return c, r


def test_planted_recovery(run0):
    c, r = run0
    inf = set(c["informative"].tolist())
    confirmed = set(np.flatnonzero(r["decision"] == 1).tolist())
    assert inf <= confirmed
    # noise is never confirmed here; most of it is rejected
    assert confirmed == inf
    assert np.sum(r["decision"] == -1) >= 12


@pytest.mark.parametrize("mode", [1, 2], ids=["permut_oob", "permut_kl"])
def test_planted_recovery_with_permutation_importances(mode):
    # both permutation importances (OOB accuracy drop, and Algorithm 3's
    # prediction divergence) confirm exactly the planted columns
    c = synth.config(0)
    pr = c["params"]
    r = O.boruta_fit(c["X"], c["y"], c["n_classes"], pr["n_trees"], pr["max_depth"],
                     importance_mode=mode, max_iter=pr["max_iter"], seed=c["seed"],
                     n_bins=pr["n_bins"])
    assert set(np.flatnonzero(r["decision"] == 1).tolist()) == set(c["informative"].tolist())
    assert np.sum(r["decision"] == -1) >= 8


def test_decisions_final_and_history(run0):
    c, r = run0
    p = c["X"].shape[1]
    prev_state = np.zeros(p, np.int8)
    prev_hits = np.zeros(p, np.int32)
    for k, tr in enumerate(r["traces"]):
        t = k + 1
        st = np.array([0] * p, np.int8)  # traces only carry integer data; rebuild from history
        row = r["imp_history"][k]
        rejected_before = prev_state == -1
        assert np.all(np.isnan(row[rejected_before]))
        assert not np.any(np.isnan(row[~rejected_before]))
        assert tr["p_cur"] == int(np.sum(prev_state >= 0))
        del st
        # recompute this iteration from (prev_state, prev_hits) with the step API
        out = O.boruta_step(c["X"], c["y"], 2, 50, 8, t=t, state=prev_state, hits=prev_hits,
                            seed=c["seed"], n_bins=64)
        assert np.array_equal(out["trace"]["imp_int"], tr["imp_int"])
        np.testing.assert_array_equal(out["imp_row"], row)
        assert out["shadow_max"] == r["shadow_max"][k]
        # decisions never change once taken; hits never exceed t
        assert np.all(out["state"][prev_state != 0] == prev_state[prev_state != 0])
        assert np.all(out["hits"] <= t)
        prev_state, prev_hits = out["state"], out["hits"]
    assert np.array_equal(prev_state, r["decision"])
    assert np.array_equal(prev_hits, r["hits"])


def test_deterministic(run0):
    c, r = run0
    r2 = O.boruta_fit(c["X"], c["y"], 2, 50, 8, max_iter=20, seed=c["seed"], n_bins=64,
                      n_threads=3)
    assert np.array_equal(r["decision"], r2["decision"])
    np.testing.assert_array_equal(r["imp_history"], r2["imp_history"])
    r3 = O.boruta_fit(c["X"], c["y"], 2, 50, 8, max_iter=20, seed=c["seed"] + 1, n_bins=64)
    assert not np.array_equal(np.nan_to_num(r["imp_history"]), np.nan_to_num(r3["imp_history"]))


@pytest.mark.parametrize("p,n_sha", [(1, 8), (2, 8), (3, 6), (4, 8), (5, 5), (7, 7)])
def test_shadow_doubling(p, n_sha):
    rng = np.random.default_rng(p)
    X = rng.standard_normal((60, p)).astype(np.float32)
    y = (X[:, 0] > 0).astype(np.int32)
    out = O.boruta_step(X, y, 2, 3, 3, t=1, state=np.zeros(p, np.int8),
                        hits=np.zeros(p, np.int32), seed=1, n_bins=16)
    tr = out["trace"]
    assert tr["n_sha"] == n_sha and tr["p_w"] == p + n_sha
    assert tr["mtry"] == int(np.floor(np.sqrt(p + n_sha)))
    assert list(tr["col_src"][p:]) == [s % p for s in range(n_sha)]


def test_stops_when_all_decided():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((300, 2)).astype(np.float32)
    y = (X[:, 0] > 0).astype(np.int32)
    X[:, 1] = rng.standard_normal(300)
    r = O.boruta_fit(X, y, 2, 20, 4, max_iter=200, seed=3, n_bins=32)
    assert r["n_iter"] < 200 and np.all(r["decision"] != 0)
    assert np.all(np.isnan(r["imp_history"][r["n_iter"]:]))


def test_mtry_clamped_and_subset_trace():
    c = synth.config(0)
    out = O.boruta_step(c["X"], c["y"], 2, 50, 8, t=1, state=np.zeros(20, np.int8),
                        hits=np.zeros(20, np.int32), mtry=1000, seed=1, n_bins=64,
                        tree_subset=[3, 17])
    tr = out["trace"]
    assert tr["mtry"] == 40
    assert set(tr["nodes"][:, 0].tolist()) == {3, 17}
    assert np.all(out["hits"] == 0)  # subset runs leave the state machine alone


def test_validation():
    X = np.zeros((10, 3), np.float32)
    y = np.zeros(10, np.int32)
    bad = [dict(n_classes=1), dict(n_classes=17), dict(alpha=0.5), dict(max_iter=0),
           dict(n_trees=0), dict(max_depth=31), dict(n_bins=257)]
    for kw in bad:
        args = dict(n_classes=2, n_trees=2, max_depth=2, alpha=0.05, max_iter=3, n_bins=8)
        args.update(kw)
        with pytest.raises(ValueError, match="-1"):
            O.boruta_fit(X, y, **args)
    y2 = y.copy()
    y2[0] = 2
    with pytest.raises(ValueError, match="-1"):
        O.boruta_fit(X, y2, 2, 2, 2)
    X2 = X.copy()
    X2[1, 1] = np.inf
    with pytest.raises(ValueError, match="-2"):
        O.boruta_fit(X2, y, 2, 2, 2)
