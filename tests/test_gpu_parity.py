"""HIP path vs CPU oracle, element by element, on seeded inputs small enough
for the oracle to finish in seconds (several histogram tiles, ragged row
counts, both node paths) and on the edge cases of the method.  Tree
structure, OOB counts, integer importances, hits and decisions must be
identical; reported importances are exactly equal."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_09950_amd import binding as B
from paper_2605_09950_amd import synth
from tests.parity_helpers import assert_same_run

pytestmark = pytest.mark.gpu


def both(X, y, K, T, D, **kw):
    kw = dict(kw)
    split_rank = kw.pop("split_rank", B.RANK_FP32)
    form = kw.pop("form", B.FORM_BATCHED)
    tune = kw.pop("tune", None)
    print(f"case n={X.shape[0]} p={X.shape[1]} K={K} T={T} D={D} {kw} rank={split_rank} "
          f"form={form} tune={tune}", flush=True)
    g = B.boruta_fit_ex(X, y, K, T, D, split_rank=split_rank, form=form, trace=True, tune=tune,
                        **kw)
    o = O.boruta_fit(X, y, K, T, D, trace=True, **kw)
    return g, o


def problem(seed, n, p, K, kind="normal"):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(np.float32)
    if kind == "mixed":
        X[:, ::3] = rng.integers(0, 4, size=X[:, ::3].shape)
        X[:, 1] = 0.25
    s = X[:, 0] + (X[:, min(1, p - 1)] > 0.3) - 0.5 * X[:, -1] + 0.5 * rng.standard_normal(n)
    y = np.digitize(s, np.quantile(s, np.linspace(0, 1, K + 1)[1:-1])).astype(np.int32)
    return X, y


@pytest.mark.parametrize("mode", [B.TREEIMP, B.PERMUT, B.PERMUT_KL])
def test_planted_small_workload(mode):
    # the small planted workload's whole run (20 iterations) in each mode
    c = synth.config(0)
    pr = c["params"]
    g, o = both(c["X"], c["y"], 2, pr["n_trees"], pr["max_depth"], max_iter=pr["max_iter"],
                seed=c["seed"], n_bins=pr["n_bins"], importance_mode=mode)
    assert_same_run(g, o)


CASES = [
    # (seed, n, p, K, T, D, extra kwargs)
    (1, 300, 7, 2, 12, 6, dict(max_iter=8, n_bins=32)),
    (2, 777, 13, 3, 9, 9, dict(max_iter=6, n_bins=256)),
    (3, 2500, 40, 4, 6, 12, dict(max_iter=4)),                    # large nodes, 2 tiles
    (4, 1200, 30, 5, 5, 8, dict(max_iter=3, mtry=20)),             # K=5 -> 8-class path
    (5, 400, 1, 2, 7, 5, dict(max_iter=10, n_bins=16)),            # p=1 -> 8 shadows
    (6, 400, 2, 3, 7, 5, dict(max_iter=10, n_bins=16)),
    (7, 400, 3, 2, 7, 5, dict(max_iter=10, n_bins=16)),            # 3 -> 6 shadows
    (8, 300, 9, 2, 8, 1, dict(max_iter=5)),                        # stumps
    (9, 600, 12, 2, 8, 7, dict(max_iter=5, n_bins=2)),             # two bins
    (10, 500, 10, 3, 8, 7, dict(max_iter=5, mtry=500)),            # mtry clamps to p_w
    (11, 900, 15, 2, 10, 10, dict(max_iter=5, kind="mixed")),      # ties, constant column
]


# histogram layouts: node-major at every level, or the column-major path from
# level 1 with runs of three items (many units per column)
PATHS = {"node": dict(col_level=64), "column": dict(col_level=1, col_unit=3)}


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", CASES, ids=[str(c[0]) for c in CASES])
def test_parity_cases(case, mode, path):
    seed, n, p, K, T, D, kw = case
    kw = dict(kw)
    X, y = problem(seed, n, p, K, kw.pop("kind", "normal"))
    extra = dict(n_perm=2) if mode == 1 else {}
    g, o = both(X, y, K, T, D, importance_mode=mode, seed=100 + seed, tune=PATHS[path],
                **extra, **kw)
    assert_same_run(g, o)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", CASES, ids=[str(c[0]) for c in CASES])
def test_plain_form_matches_oracle(case, mode):
    # the plain form (one launch per tree node: histogram, then split and
    # partition, per large node) against the oracle directly
    seed, n, p, K, T, D, kw = case
    kw = dict(kw)
    X, y = problem(seed, n, p, K, kw.pop("kind", "normal"))
    extra = dict(n_perm=2) if mode == 1 else {}
    g, o = both(X, y, K, T, D, importance_mode=mode, seed=200 + seed, form=B.FORM_PLAIN,
                **extra, **kw)
    assert_same_run(g, o)


def test_many_classes_and_tiny_n():
    X, y = problem(12, 3000, 20, 16)
    for tune in PATHS.values():
        g, o = both(X, y, 16, 4, 10, max_iter=3, seed=3, tune=tune)
        assert_same_run(g, o)
    rng = np.random.default_rng(0)
    for n in (2, 3, 5):
        X = rng.standard_normal((n, 4)).astype(np.float32)
        y = (np.arange(n) % 2).astype(np.int32)
        for mode in (0, 1):
            g, o = both(X, y, 2, 5, 3, max_iter=4, seed=n, importance_mode=mode)
            assert_same_run(g, o)


@pytest.mark.parametrize("mode", [0, 1])
def test_exact_and_fp32_ranking_give_identical_runs(mode):
    X, y = problem(21, 3000, 60, 3)
    kw = dict(importance_mode=mode, max_iter=4, seed=5, trace=True)
    a = B.boruta_fit_ex(X, y, 3, 10, 10, split_rank=B.RANK_EXACT, **kw)
    b = B.boruta_fit_ex(X, y, 3, 10, 10, split_rank=B.RANK_FP32, **kw)
    assert_same_run(a, b)


def test_plain_and_batched_forms_identical():
    X, y = problem(22, 1500, 25, 3)
    kw = dict(max_iter=3, seed=6, trace=True)
    a = B.boruta_fit_ex(X, y, 3, 6, 8, form=B.FORM_PLAIN, **kw)
    b = B.boruta_fit_ex(X, y, 3, 6, 8, form=B.FORM_BATCHED, **kw)
    assert_same_run(a, b)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_batch_mixing_class_counts_matches_oracle(path):
    # jobs of 2, 3 and 4 classes beside one of 6 (8 class planes for the
    # batch): the small-class jobs' node-major items take the 4-plane kernel
    jobs = []
    for j, K in enumerate((2, 6, 3, 4)):
        X, y = problem(60 + j, 900 + 400 * j, 18, K)
        jobs.append(dict(X=X, y=y, n_classes=K, n_trees=5, max_depth=9, importance_mode=j % 2,
                         max_iter=3, seed=70 + j))
    print(f"mixed-class batch, path {path}", flush=True)
    batch = B.boruta_fit_batch(jobs, trace=True, tune=PATHS[path])
    for j, jd in enumerate(jobs):
        o = O.boruta_fit(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"], jd["max_depth"],
                         importance_mode=jd["importance_mode"], max_iter=jd["max_iter"],
                         seed=jd["seed"], trace=True)
        r = dict(batch["results"][j])
        r["traces"] = [t for t in batch["traces"] if t["job"] == j]
        assert r["status"] == 0
        assert_same_run(r, o)


def test_batch_of_long_and_short_jobs_matches_oracle():
    # bootstrap multiplicities of n = 70,001 rows are counted in three row
    # chunks (every chunk evaluates all draws), beside a job of 3,000 rows in
    # the same launches
    jobs = []
    for j, (n, K) in enumerate(((70001, 2), (3000, 3))):
        X, y = problem(80 + j, n, 6, K)
        jobs.append(dict(X=X, y=y, n_classes=K, n_trees=3, max_depth=5, max_iter=2, seed=90 + j))
    batch = B.boruta_fit_batch(jobs, trace=True)
    for j, jd in enumerate(jobs):
        o = O.boruta_fit(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"], jd["max_depth"],
                         max_iter=jd["max_iter"], seed=jd["seed"], trace=True)
        r = dict(batch["results"][j])
        r["traces"] = [t for t in batch["traces"] if t["job"] == j]
        assert r["status"] == 0
        assert_same_run(r, o)


def test_job_beyond_the_lds_bootstrap_counts_matches_oracle():
    # n = 140,000 rows: more than the LDS row chunks cover, so the bootstrap
    # multiplicities take the global-atomic kernel
    X, y = problem(85, 140000, 5, 2)
    kw = dict(max_iter=2, seed=11)
    print("n = 140,000 bootstrap by global atomics", flush=True)
    g, o = both(X, y, 2, 3, 4, **kw)
    assert_same_run(g, o)


def test_batch_equals_single_jobs():
    jobs = []
    for j in range(6):
        X, y = problem(30 + j, 200 + 300 * j, 15, 2 + j % 3)
        jobs.append(dict(X=X, y=y, n_classes=2 + j % 3, n_trees=4 + j, max_depth=6 + j,
                         importance_mode=j % 3, max_iter=3 + j, seed=40 + j))
    batch = B.boruta_fit_batch(jobs, trace=True)
    for j, jd in enumerate(jobs):
        single = B.boruta_fit_ex(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"],
                                 jd["max_depth"], importance_mode=jd["importance_mode"],
                                 max_iter=jd["max_iter"], seed=jd["seed"], trace=True)
        r = dict(batch["results"][j])
        r["traces"] = [t for t in batch["traces"] if t["job"] == j]
        assert r["status"] == 0
        assert_same_run(r, single)


def test_batch_jobs_sharing_inputs_equal_single_jobs():
    # jobs passing the same X and y arrays are binned once and share the binned
    # matrix; each still equals its own single run (mixed with an unshared job,
    # and with a job of the same arrays but another importance mode)
    X, y = problem(33, 900, 13, 3)
    X2, y2 = problem(34, 700, 9, 2)
    jobs = [dict(X=X, y=y, n_classes=3, n_trees=6, max_depth=8, max_iter=5, seed=s)
            for s in (1, 2)]
    jobs.insert(1, dict(X=X2, y=y2, n_classes=2, n_trees=5, max_depth=7, max_iter=4, seed=3))
    jobs.append(dict(X=X, y=y, n_classes=3, n_trees=7, max_depth=9, importance_mode=B.PERMUT,
                     max_iter=4, seed=4))
    batch = B.boruta_fit_batch(jobs, trace=True)
    for j, jd in enumerate(jobs):
        single = B.boruta_fit_ex(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"],
                                 jd["max_depth"], importance_mode=jd.get("importance_mode", 0),
                                 max_iter=jd["max_iter"], seed=jd["seed"], trace=True)
        r = dict(batch["results"][j])
        r["traces"] = [t for t in batch["traces"] if t["job"] == j]
        assert r["status"] == 0
        assert_same_run(r, single)
    # a shared input that fails validation fails every job that shares it
    Xbad = X.copy()
    Xbad[5, 2] = np.nan
    bad = [dict(jobs[0], X=Xbad), dict(jobs[2], X=Xbad)]
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_batch(bad)
    assert e.value.code == B.BORUTA_E_NONFINITE


def test_allocation_failure_returns_oom_and_leaks_nothing(monkeypatch):
    # the failure hook makes the library's device allocation fail: every entry
    # point that allocates returns BORUTA_E_OOM, device memory does not
    # shrink over repeated failures, and later calls give the usual results
    import torch
    X, y = problem(24, 700, 9, 2)
    kw = dict(max_iter=3, seed=5)
    want = B.boruta_fit_ex(X, y, 2, 5, 7, **kw)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    monkeypatch.setenv("BORUTA_FAIL_ALLOC", "1")
    calls = [lambda: B.boruta_fit_ex(X, y, 2, 5, 7, **kw),
             lambda: B.boruta_fit_batch([dict(X=X, y=y, n_classes=2, n_trees=5, max_depth=7,
                                              **kw)]),
             lambda: B.boruta_fit_seeds(X, y, 2, 5, 7, [1, 2], max_iter=3),
             lambda: B.boruta_fit_regression(X, X[:, 0].copy(), 5, 7, **kw),
             lambda: B.Session([dict(X=X, y=y, n_classes=2, n_trees=5, max_depth=7, **kw)])]
    for _ in range(5):
        for call in calls:
            with pytest.raises(B.BorutaError) as e:
                call()
            assert e.value.code == B.BORUTA_E_OOM
    monkeypatch.delenv("BORUTA_FAIL_ALLOC")
    torch.cuda.synchronize()
    assert free0 - torch.cuda.mem_get_info()[0] < (16 << 20)
    again = B.boruta_fit_ex(X, y, 2, 5, 7, **kw)
    assert np.array_equal(again["decision"], want["decision"])
    assert np.array_equal(again["imp_history"], want["imp_history"], equal_nan=True)


@pytest.mark.parametrize("n,n_bins", [(1, 2), (300, 16), (1000, 256), (70000, 256)],
                         ids=["n1", "n300_b16", "n1000", "n70000"])
def test_device_binning_equals_oracle_bins(n, n_bins):
    # the binning step alone: every byte against the oracle's bins (ragged n,
    # several sort tiles at n = 70000, ties, categorical codes, a constant
    # column, signed zeros, heavy tails)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 7)).astype(np.float32)
    X[:, 1] = rng.integers(0, 5, n)
    X[:, 2] = 1.5
    X[:, 3] = np.where(rng.random(n) < 0.5, -0.0, 0.0)
    X[:, 4] = np.round(X[:, 4], 1)
    X[:, 5] = np.exp(3 * X[:, 5])
    print(f"binning n={n} p=7 bins={n_bins}", flush=True)
    got = B.boruta_bin(X, n_bins)
    want, _, _ = O.bin_matrix(X, n_bins)
    assert np.array_equal(got, want)
    X[n // 2, 6] = np.nan
    with pytest.raises(B.BorutaError) as e:
        B.boruta_bin(X, n_bins)
    assert e.value.code == B.BORUTA_E_NONFINITE


def test_device_entry_point_matches_host_entry_point():
    import torch
    X, y = problem(23, 1000, 12, 2)
    ws = B.boruta_workspace_size([dict(n=1000, p=12, n_classes=2, n_trees=8, max_depth=8,
                                       max_iter=5)])
    dX = torch.from_numpy(X).cuda()
    dy = torch.from_numpy(y).cuda()
    w = torch.empty(ws, dtype=torch.uint8, device="cuda")
    d = B.boruta_fit_device(dX, dy, 2, 8, 8, w, max_iter=5, seed=9, trace=True)
    h = B.boruta_fit_ex(X, y, 2, 8, 8, max_iter=5, seed=9, trace=True)
    assert_same_run(d, h)
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_device(dX, dy, 2, 8, 8, w[: ws // 2], max_iter=5, seed=9)
    assert e.value.code == B.BORUTA_E_OOM


def test_nonfinite_and_bad_labels_detected_on_device():
    X, y = problem(24, 100, 4, 2)
    X[7, 2] = np.inf
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_ex(X, y, 2, 3, 3)
    assert e.value.code == B.BORUTA_E_NONFINITE
    X, y = problem(24, 100, 4, 2)
    y[3] = 2
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_ex(X, y, 2, 3, 3)
    assert e.value.code == B.BORUTA_E_INVALID_ARG


def test_session_steps_and_resume_reproduce_a_run():
    X, y = problem(25, 800, 14, 3)
    kw = dict(n_classes=3, n_trees=6, max_depth=7, max_iter=12, seed=11)
    full = B.boruta_fit_ex(X, y, 3, 6, 7, max_iter=12, seed=11)
    with B.Session([dict(X=X, y=y, **kw)]) as s:
        for _ in range(5):
            s.step()
        mid = s.result(0)
        while s.step():
            pass
        end = s.result(0)
    assert mid["n_iter"] == 5
    for key in ("decision", "hits", "n_iter"):
        assert np.array_equal(np.asarray(end[key]), np.asarray(full[key]))
    k = full["n_iter"]
    np.testing.assert_array_equal(end["imp_history"][:k], full["imp_history"][:k])
    # a fresh session resumed from the iteration-5 checkpoint finishes identically
    with B.Session([dict(X=X, y=y, **kw)]) as s:
        s.resume(0, 5, mid["decision"], mid["hits"])
        while s.step():
            pass
        res = s.result(0)
    assert np.array_equal(res["decision"], full["decision"])
    assert np.array_equal(res["hits"], full["hits"])
    assert res["n_iter"] == full["n_iter"]
    np.testing.assert_array_equal(res["imp_history"][5:k], full["imp_history"][5:k])


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_graph_replays_match_eager_launches(mode):
    """The batched iteration captured once as a HIP graph and replayed every
    step (with the host's read-back and checks between replays) gives the
    eager launch sequence's run, iteration by iteration."""
    X, y = problem(26, 1800, 24, 3)
    kw = dict(importance_mode=mode, max_iter=7, seed=12, trace=True)
    eager = B.boruta_fit_ex(X, y, 3, 8, 9, graph=False, **kw)
    graph = B.boruta_fit_ex(X, y, 3, 8, 9, graph=True, **kw)
    assert len(graph["traces"]) >= 3
    assert_same_run(graph, eager)


@pytest.mark.parametrize("chunk", [100, 3])
def test_session_run_back_to_back_equals_stepping(chunk):
    # iterations enqueued back to back (graph replays without host waits), for
    # a batch whose jobs finish at different iterations: the same results as
    # one step at a time, and the job-iterations counted on the device
    jobs = []
    for j in range(4):
        X, y = problem(80 + j, 500 + 200 * j, 9 + j, 2 + j % 2)
        jobs.append(dict(X=X, y=y, n_classes=2 + j % 2, n_trees=6, max_depth=7,
                         importance_mode=j % 3, max_iter=3 + 3 * j, seed=90 + j))
    with B.Session(jobs) as a:
        while a.step():
            pass
        want = [a.result(j) for j in range(len(jobs))]
    total = 0
    with B.Session(jobs) as b:
        live = len(jobs)
        while live:
            live, done = b.run(chunk)
            total += done
        got = [b.result(j) for j in range(len(jobs))]
        assert b.run(5) == (0, 0)  # nothing left to run
    assert total == sum(w["n_iter"] for w in want)
    for g, w in zip(got, want):
        assert g["n_iter"] == w["n_iter"]
        assert np.array_equal(g["decision"], w["decision"])
        assert np.array_equal(g["hits"], w["hits"])
        assert np.array_equal(g["rank"], w["rank"])
        k = w["n_iter"]
        assert np.array_equal(g["imp_history"][:k], w["imp_history"][:k], equal_nan=True)


def test_permutation_node_visits_counted_under_statistics():
    # every OOB row walks at least its root; a walk of depth <= D visits at
    # most D + 1 nodes, and each of at most D path columns is re-routed R times
    X, y = problem(29, 800, 12, 2)
    R, D = 2, 7
    jd = dict(X=X, y=y, n_classes=2, n_trees=5, max_depth=D, max_iter=3, seed=21)
    with B.Session([dict(jd, importance_mode=B.PERMUT)], n_perm=R, stats=True,
                   trace=True) as s:
        while s.step():
            pass
        v = s.stats.permut_visits
        m = sum(int(t["tree_stats"][:, 2].sum()) for t in s.traces)
    assert m > 0 and m <= v <= m * (D + 1) * (1 + R * D)
    with B.Session([dict(jd, importance_mode=B.TREEIMP)], stats=True) as s:
        while s.step():
            pass
        assert s.stats.permut_visits == 0


def test_graph_session_with_stats_and_resume():
    X, y = problem(27, 900, 16, 2)
    kw = dict(n_classes=2, n_trees=7, max_depth=8, max_iter=10, seed=13)
    full = B.boruta_fit_ex(X, y, 2, 7, 8, max_iter=10, seed=13, graph=False)
    with B.Session([dict(X=X, y=y, **kw)], stats=True, graph=True) as s:
        for _ in range(4):
            s.step()
        mid = s.result(0)
        st = s.stats
        assert st.iterations == 4 and st.hist_small.launches == 4 * 8
        assert st.iter_ms > 0 and st.hist_large.ms > 0
    with B.Session([dict(X=X, y=y, **kw)], graph=True) as s:
        s.resume(0, 4, mid["decision"], mid["hits"])
        while s.step():
            pass
        res = s.result(0)
    assert np.array_equal(res["decision"], full["decision"])
    assert np.array_equal(res["hits"], full["hits"])
    k = full["n_iter"]
    assert res["n_iter"] == k
    np.testing.assert_array_equal(res["imp_history"][4:k], full["imp_history"][4:k])


@pytest.mark.parametrize("K", [2, 4])
@pytest.mark.parametrize("tune", [dict(small_rows=16), dict(small_rows=64),
                                  dict(small_rows=32, grid_hist=64, grid_small=8,
                                       grid_finalize=3),
                                  dict(col_level=64),
                                  dict(col_level=1, col_unit=1, grid_col=5),
                                  dict(col_level=3, col_unit=7, grid_col=64)],
                         ids=["small_rows16", "small_rows64", "tiny_grids", "node_major_only", "column_all_tiny",
                              "column_from3"])
def test_launch_tuning_leaves_results_unchanged(tune, K):
    X, y = problem(28, 2200, 30, K)
    kw = dict(max_iter=4, seed=14, trace=True)
    a = B.boruta_fit_ex(X, y, K, 8, 10, **kw)
    b = B.boruta_fit_ex(X, y, K, 8, 10, tune=tune, **kw)
    assert_same_run(a, b)


@pytest.mark.parametrize("split_rank", [B.RANK_FP32, B.RANK_EXACT], ids=["fp32", "exact"])
@pytest.mark.parametrize("K", [2, 3, 4])
def test_wide_small_node_segments_match_oracle(K, split_rank):
    # nodes of up to 64 rows on the wave path: segments of 32 and 64 lanes
    # score their thresholds in the sorted form
    X, y = problem(91 + K, 1800, 24, K, kind="mixed")
    g, o = both(X, y, K, 10, 11, max_iter=5, seed=23, split_rank=split_rank,
                tune=dict(small_rows=64))
    assert_same_run(g, o)


def test_final_ranking_matches_oracle():
    # Algorithm 1's ranking through the batch API (all three importance
    # modes) and through a session's result
    jobs = []
    for j in range(3):
        X, y = problem(50 + j, 600, 14, 3)
        jobs.append(dict(X=X, y=y, n_classes=3, n_trees=8, max_depth=7, importance_mode=j,
                         max_iter=12, seed=60 + j))
    batch = B.boruta_fit_batch(jobs)
    for j, jd in enumerate(jobs):
        o = O.boruta_fit(jd["X"], jd["y"], 3, 8, 7, importance_mode=j, max_iter=12, seed=60 + j)
        r = batch["results"][j]
        assert r["n_iter"] == o["n_iter"]
        assert np.array_equal(r["decision"], o["decision"])
        assert np.array_equal(r["rank"], o["rank"])
        assert (r["rank"] == 3).any() or not (r["decision"] == -1).any()
    with B.Session(jobs[:1]) as s:
        while s.step():
            pass
        assert np.array_equal(s.result(0)["rank"], batch["results"][0]["rank"])


@pytest.mark.parametrize("seeds", [[3, 11, 29, 47, 90], [5, 6, 7, 8]], ids=["odd", "even"])
def test_multi_seed_median_matches_oracle(seeds):
    # the repeated-seed protocol: every run against the oracle's run of its
    # seed, and the device aggregate against the oracle's aggregate of those
    # runs (an odd count takes the middle value, an even one the mean of two)
    X, y = problem(77, 700, 16, 2)
    kw = dict(mtry=0, importance_mode=B.PERMUT, max_iter=10, alpha=0.05)
    print(f"multi-seed n=700 p=16 seeds={seeds}", flush=True)
    g = B.boruta_fit_seeds(X, y, 2, 8, 8, seeds, **kw)
    runs = []
    for i, sd in enumerate(seeds):
        o = O.boruta_fit(X, y, 2, 8, 8, seed=sd, **kw)
        r = g["runs"][i]
        assert r["n_iter"] == o["n_iter"]
        assert np.array_equal(r["decision"], o["decision"])
        assert np.array_equal(r["imp_history"], o["imp_history"], equal_nan=True)
        runs.append(o)
    med, dec = O.seed_median(runs)
    assert np.array_equal(g["median_importance"], med)
    assert np.array_equal(g["decision"], dec)
    # without per-run outputs the aggregate is the same
    h = B.boruta_fit_seeds(X, y, 2, 8, 8, seeds, runs=False, **kw)
    assert np.array_equal(h["median_importance"], med)
    assert np.array_equal(h["decision"], dec)
    assert (dec == 1).any()
    Xbad = X.copy()
    Xbad[3, 1] = np.inf
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_seeds(Xbad, y, 2, 8, 8, seeds[:2], **kw)
    assert e.value.code == B.BORUTA_E_NONFINITE


@pytest.mark.parametrize("perc", [90, 50])
@pytest.mark.parametrize("mode", [B.TREEIMP, B.PERMUT, B.PERMUT_KL])
def test_percentile_shadow_threshold_matches_oracle(mode, perc):
    # the hit threshold as the perc-th percentile of the shadow importances
    # (radix select on the device)
    X, y = problem(61, 900, 14, 3)
    kw = dict(importance_mode=mode, max_iter=8, seed=31, perc=perc)
    g, o = both(X, y, 3, 8, 8, **kw)
    assert_same_run(g, o)
    assert (g["hits"] > 0).any()


@pytest.mark.parametrize("perc", [1, 37, 99])
def test_percentile_threshold_over_many_shadows(perc):
    # ~600 shadow columns (several candidates per radix digit) and Permut's
    # signed importances (negative keys)
    X, y = problem(62, 400, 600, 2)
    g, o = both(X, y, 2, 6, 6, importance_mode=B.PERMUT, max_iter=2, seed=32, perc=perc)
    assert_same_run(g, o)


def test_rough_fix_matches_oracle_and_leaves_the_session_state():
    # tentative features resolved by the rough fix in the reported decision
    # and rank (batch of two modes; multi-seed aggregate); a session read
    # mid-run with the fix continues exactly like one read without it
    X, y = problem(63, 800, 12, 2)
    jobs = [dict(X=X, y=y, n_classes=2, n_trees=8, max_depth=8, importance_mode=m, max_iter=9,
                 seed=70 + m) for m in (0, 1)]
    batch = B.boruta_fit_batch(jobs, rough_fix=True)
    for j, jd in enumerate(jobs):
        o = O.boruta_fit(X, y, 2, 8, 8, importance_mode=jd["importance_mode"], max_iter=9,
                         seed=jd["seed"], rough_fix=True)
        r = batch["results"][j]
        assert np.array_equal(r["decision"], o["decision"])
        assert np.array_equal(r["rank"], o["rank"])
        assert not (r["decision"] == 0).any()
    plain = B.boruta_fit_batch(jobs)
    assert any((r["decision"] == 0).any() for r in plain["results"])
    seeds = [5, 6, 7]
    g = B.boruta_fit_seeds(X, y, 2, 8, 8, seeds, max_iter=9, rough_fix=True)
    runs = [O.boruta_fit(X, y, 2, 8, 8, max_iter=9, seed=s, rough_fix=True) for s in seeds]
    med, dec = O.seed_median(runs)
    assert np.array_equal(g["median_importance"], med)
    assert np.array_equal(g["decision"], dec)
    with B.Session(jobs[:1], rough_fix=True) as s:
        for _ in range(4):
            s.step()
        mid = s.result(0)
        o4 = O.boruta_fit(X, y, 2, 8, 8, max_iter=4, seed=70, rough_fix=True)
        assert np.array_equal(mid["decision"], o4["decision"])
        while s.step():
            pass
        assert np.array_equal(s.result(0)["decision"], batch["results"][0]["decision"])


@pytest.mark.parametrize("kl_rows", [7, 256])
def test_kl_importance_in_row_blocks(kl_rows):
    # the divergence step in blocks of 7 rows (ragged last block) or 256,
    # against the oracle, and against the default single block
    X, y = problem(41, 1500, 12, 3)
    kw = dict(importance_mode=2, max_iter=4, seed=17)
    g, o = both(X, y, 3, 9, 9, tune=dict(kl_rows=kl_rows), **kw)
    assert_same_run(g, o)
    d = B.boruta_fit_ex(X, y, 3, 9, 9, trace=True, **kw)
    assert_same_run(g, d)


def test_kl_importance_medium_problem():
    X, y = problem(42, 4000, 40, 4, "mixed")
    g, o = both(X, y, 4, 24, 12, importance_mode=2, max_iter=3, seed=18)
    assert_same_run(g, o)


def test_autotuner_returns_a_valid_choice(tmp_path):
    from paper_2605_09950_amd import autotune as A
    c = synth.config(0)
    pr = c["params"]
    jobs = [dict(X=c["X"], y=c["y"], n_classes=2, n_trees=pr["n_trees"],
                 max_depth=pr["max_depth"], max_iter=pr["max_iter"], seed=c["seed"])]
    cache = str(tmp_path / "tune.json")
    t = A.autotune(jobs, n_bins=pr["n_bins"], steps=1, warmup=1, cache=cache)
    assert set(t) <= set(B.TUNE_KEYS)
    assert A.autotune(jobs, n_bins=pr["n_bins"], cache=cache) == t  # served from the cache
    g = B.boruta_fit_ex(c["X"], c["y"], 2, pr["n_trees"], pr["max_depth"], max_iter=4,
                        seed=c["seed"], n_bins=pr["n_bins"], tune=t)
    d = B.boruta_fit_ex(c["X"], c["y"], 2, pr["n_trees"], pr["max_depth"], max_iter=4,
                        seed=c["seed"], n_bins=pr["n_bins"])
    assert_same_run(g, d)
