"""HIP path vs CPU oracle for the regression forest (float targets held as
exact fixed point, squared-error splits, all three importance modes): tree
structure (a leaf's prediction floor(T / W) in the trace), in-bag / OOB
counts, integer importances, hits, decisions and reported importances are
identical."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_09950_amd import binding as B
from tests.parity_helpers import assert_same_run

pytestmark = pytest.mark.gpu


def problem(seed, n, p, kind="smooth"):
    rng = np.random.default_rng(seed)
    X = rng.random((n, p)).astype(np.float32)
    y = 3 * X[:, 0] + 2 * np.sin(4 * X[:, 1]) + (X[:, 2] > 0.6) + 0.4 * rng.standard_normal(n)
    if kind == "ties":  # few distinct targets: equal scores between thresholds
        y = np.round(y)
    if kind == "outlier":  # one far target: the others use few fixed-point bits
        y[rng.integers(0, n)] = 40.0
    if kind == "wide":  # negative targets over 60 binades, many rounded in fixed point
        y = (y - 2.5) * np.exp(rng.uniform(-40, 0, n))
    return X, y.astype(np.float32)


def both(X, y, T, D, **kw):
    kw = dict(kw)
    split_rank = kw.pop("split_rank", B.RANK_FP32)
    tune = kw.pop("tune", None)
    print(f"regression n={X.shape[0]} p={X.shape[1]} T={T} D={D} {kw} rank={split_rank} "
          f"tune={tune}", flush=True)
    g = B.boruta_fit_regression(X, y, T, D, split_rank=split_rank, trace=True, tune=tune, **kw)
    o = O.boruta_fit_reg(X, y, T, D, trace=True, **kw)
    return g, o


@pytest.mark.parametrize("split_rank", [B.RANK_FP32, B.RANK_EXACT], ids=["fp32", "exact"])
@pytest.mark.parametrize("kind", ["smooth", "ties", "outlier", "wide"])
def test_regression_run_matches_oracle(kind, split_rank):
    X, y = problem(41, 900, 11, kind)
    g, o = both(X, y, 9, 9, max_iter=6, seed=12, split_rank=split_rank)
    assert_same_run(g, o)
    assert len(g["traces"]) == g["n_iter"]


@pytest.mark.parametrize("n_perm", [1, 3])
@pytest.mark.parametrize("kind", ["smooth", "ties"])
def test_regression_permutation_importance_matches_oracle(kind, n_perm):
    # out-of-bag squared-error increase under column permutation
    X, y = problem(47, 1000, 10, kind)
    g, o = both(X, y, 8, 9, importance_mode=B.PERMUT, max_iter=6, seed=16, n_perm=n_perm)
    assert_same_run(g, o)
    assert (g["hits"] > 0).any()


@pytest.mark.parametrize("kl_rows", [0, 7])
def test_regression_divergence_importance_matches_oracle(kl_rows):
    # Algorithm 3 for regression: squared difference of the mean predictions
    # under the shared row permutation (one row block, or blocks of 7 rows)
    X, y = problem(49, 900, 10)
    g, o = both(X, y, 8, 9, importance_mode=B.PERMUT_KL, max_iter=5, seed=18,
                tune=dict(kl_rows=kl_rows) if kl_rows else None)
    assert_same_run(g, o)
    assert (g["hits"] > 0).any()


def test_regression_permutation_importance_many_columns():
    # more columns than the per-workgroup drop sums hold: the path that adds
    # every row's drop to the importances directly, as regression always does
    X, y = problem(48, 700, 600)
    g, o = both(X, y, 4, 8, importance_mode=B.PERMUT, max_iter=2, seed=17, n_bins=32)
    assert_same_run(g, o)


@pytest.mark.parametrize("tune", [dict(small_rows=16), dict(small_rows=64),
                                  dict(col_level=1, col_unit=3), dict(col_level=64)],
                         ids=["small16", "small64", "column", "node_major"])
def test_regression_launch_paths_match_oracle(tune):
    X, y = problem(42, 2500, 20)
    g, o = both(X, y, 7, 12, max_iter=4, seed=13, n_bins=64, tune=tune)
    assert_same_run(g, o)


def test_regression_recovers_planted_features_like_the_oracle():
    X, y = problem(43, 3000, 16)
    g, o = both(X, y, 30, 10, max_iter=25, seed=14)
    assert_same_run(g, o)
    assert list(g["decision"][:3]) == [1, 1, 1]


def test_constant_target_grows_stumps():
    X, _ = problem(44, 300, 6)
    y = np.full(300, 2.5, np.float32)
    g, o = both(X, y, 5, 6, max_iter=3, seed=15)
    assert_same_run(g, o)
    assert (g["hits"] == 0).all()
    for tr in g["traces"]:
        assert (tr["nodes"][:, 2] == -1).all()  # every tree is a single leaf


def test_regression_jobs_in_a_batch_and_a_device_session():
    # a regression job beside a classification job in one batch, and a session
    # over device-resident inputs: each equals its own single run
    import torch
    Xr, yr = problem(45, 1200, 9)
    rng = np.random.default_rng(46)
    Xc = rng.standard_normal((800, 7)).astype(np.float32)
    yc = (Xc[:, 0] > 0).astype(np.int32)
    jobs = [dict(X=Xr, y_reg=yr, n_trees=6, max_depth=9, max_iter=4, seed=3),
            dict(X=Xc, y=yc, n_classes=2, n_trees=5, max_depth=7, max_iter=4, seed=4)]
    batch = B.boruta_fit_batch(jobs, trace=True)
    reg = B.boruta_fit_regression(Xr, yr, 6, 9, max_iter=4, seed=3, trace=True)
    cls = B.boruta_fit_ex(Xc, yc, 2, 5, 7, max_iter=4, seed=4, trace=True)
    for j, single in enumerate((reg, cls)):
        r = dict(batch["results"][j])
        r["traces"] = [t for t in batch["traces"] if t["job"] == j]
        assert r["status"] == 0
        assert_same_run(r, single)
    dev = [dict(X=torch.from_numpy(Xr).cuda(), y_reg=torch.from_numpy(yr).cuda(), n_trees=6,
                max_depth=9, max_iter=4, seed=3)]
    ws_bytes = B.boruta_workspace_size([dict(n=1200, p=9, n_classes=2, n_trees=6, max_depth=9,
                                             max_iter=4, regression=True)])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    with B.Session(dev, inputs_on_device=True, workspace=ws,
                   stream=torch.cuda.current_stream()) as s:
        while s.step():
            pass
        res = s.result(0)
    assert res["n_iter"] == reg["n_iter"]
    assert np.array_equal(res["decision"], reg["decision"])
    k = reg["n_iter"]
    assert np.array_equal(res["imp_history"][:k], reg["imp_history"][:k])


@pytest.mark.parametrize("n,p,D", [(2, 1, 1), (3, 2, 3), (5, 1, 30)], ids=["n2p1", "n3p2", "n5p1D30"])
def test_regression_degenerate_shapes(n, p, D):
    # two to five rows, one or two features (shadow doubling), depth 1 and 30
    rng = np.random.default_rng(50 + n)
    X = rng.random((n, p)).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    for mode in (B.TREEIMP, B.PERMUT, B.PERMUT_KL):
        g, o = both(X, y, 3, D, importance_mode=mode, max_iter=3, seed=19)
        assert_same_run(g, o)


def test_regression_past_65536_rows():
    # n = 100,000: the fixed-point sums have no row cap short of n <= 2^24
    rng = np.random.default_rng(51)
    n, p = 100000, 4
    X = rng.random((n, p)).astype(np.float32)
    y = (X[:, 0] + 0.1 * rng.standard_normal(n)).astype(np.float32)
    for mode in (B.TREEIMP, B.PERMUT):
        g, o = both(X, y, 3, 6, importance_mode=mode, max_iter=2, seed=20, n_bins=64)
        assert_same_run(g, o)
        root_w = max(int(t["nodes"][t["nodes"][:, 1] == 1, 4].max()) for t in g["traces"])
        assert root_w == n  # the root's bootstrap weight: the n draws


def test_regression_plain_per_node_form_matches_oracle():
    # the plain form (one launch per tree node)
    X, y = problem(52, 400, 7)
    g = B.boruta_fit_regression(X, y, 4, 6, max_iter=3, seed=21, form=B.FORM_PLAIN, trace=True)
    o = O.boruta_fit_reg(X, y, 4, 6, max_iter=3, seed=21, trace=True)
    assert_same_run(g, o)


def test_regression_multi_seed_median_matches_oracle():
    # the paper's repeated-seed protocol on a regression problem
    X, y = problem(53, 600, 8)
    seeds = [4, 9, 13]
    g = B.boruta_fit_seeds(X, y, None, 6, 8, seeds, importance_mode=B.PERMUT, max_iter=6)
    runs = [O.boruta_fit_reg(X, y, 6, 8, importance_mode=1, max_iter=6, seed=s) for s in seeds]
    for r, o in zip(g["runs"], runs):
        assert r["n_iter"] == o["n_iter"]
        assert np.array_equal(r["decision"], o["decision"])
    med, dec = O.seed_median(runs)
    assert np.array_equal(g["median_importance"], med)
    assert np.array_equal(g["decision"], dec)
