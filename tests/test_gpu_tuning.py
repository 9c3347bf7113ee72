"""Launch tuning on the GPU: every histogram shape (rows per lane per batch
for the shallow and the deep tree levels and their boundary, drawn features
per item, wavefronts per workgroup of the column-major kernel) gives the
oracle's run, and the library applies a tuning cache file written by the
autotuner (boruta_options.tune_cache) to the fields its caller left at their
defaults."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_09950_amd import autotune as A
from paper_2605_09950_amd import binding as B
from tests.parity_helpers import assert_same_run

pytestmark = pytest.mark.gpu


def problem(seed, n, p, K):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(np.float32)
    X[:, 3] = np.round(X[:, 3] * 2)  # a column with few distinct values
    y = np.argmax(X[:, :K] + 0.7 * rng.standard_normal((n, K)), axis=1).astype(np.int32)
    return X, y


SHAPES = [dict(hist_rb=4), dict(hist_rb=16), dict(hist_rb_deep=4, band_level=2),
          dict(hist_rb=16, hist_rb_deep=4, band_level=3), dict(hist_fw=1), dict(hist_fw=2),
          dict(hist_fw=4), dict(col_level=2, col_unit=5, col_waves=2),
          dict(col_level=1, col_waves=7)]


@pytest.mark.parametrize("K", [2, 3])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda d: ",".join(f"{k}{v}" for k, v in d.items()))
def test_every_histogram_shape_matches_the_oracle(shape, K):
    X, y = problem(71 + K, 2600, 24, K)
    kw = dict(max_iter=4, seed=90 + K, n_bins=64)
    print(f"shape {shape} K={K}", flush=True)
    g = B.boruta_fit_ex(X, y, K, 7, 9, trace=True, tune=shape, **kw)
    o = O.boruta_fit(X, y, K, 7, 9, trace=True, **kw)
    assert_same_run(g, o)


def test_regression_with_every_fw_matches_the_oracle():
    # a regression job needs 768 LDS words per wavefront: one draw per item
    # with two class planes is raised to two draws
    rng = np.random.default_rng(75)
    X = rng.random((1500, 12)).astype(np.float32)
    y = (3 * X[:, 0] + np.sin(5 * X[:, 1]) + 0.3 * rng.standard_normal(1500)).astype(np.float32)
    o = O.boruta_fit_reg(X, y, 5, 8, max_iter=3, seed=4, trace=True)
    for fw in (1, 2, 4):
        g = B.boruta_fit_regression(X, y, 5, 8, max_iter=3, seed=4, trace=True,
                                    tune=dict(hist_fw=fw, hist_rb=4))
        assert_same_run(g, o)


def test_tuning_cache_is_applied_by_the_library(tmp_path):
    X, y = problem(77, 2000, 20, 3)
    jd = dict(X=X, y=y, n_classes=3, n_trees=6, max_depth=8, mtry=0, importance_mode=0,
              max_iter=3, seed=5)
    cache = str(tmp_path / "tune.txt")
    sig = A.signature([jd], n_bins=64, n_perm=1)
    A.write_cache(cache, {sig: dict(col_level=2, col_unit=7, hist_rb=4, hist_fw=1),
                          "B64|R1|1x1K2T1D1m0i0": dict(col_level=1)})
    kw = dict(max_iter=3, seed=5, n_bins=64)
    base = B.boruta_fit_ex(X, y, 3, 6, 8, stats=True, **kw)
    assert base["stats"].hist_col.launches == 0  # node-major at every level by default
    cached = B.boruta_fit_ex(X, y, 3, 6, 8, stats=True, tune=dict(tune_cache=cache), **kw)
    # the cache's col_level = 2 put levels 2..7 on the column-major path
    assert cached["stats"].hist_col.launches > 0
    for k in ("decision", "hits", "shadow_max"):
        assert np.array_equal(base[k], cached[k], equal_nan=True)
    # a value the caller sets wins over the cache
    own = B.boruta_fit_ex(X, y, 3, 6, 8, stats=True,
                          tune=dict(tune_cache=cache, col_level=64), **kw)
    assert own["stats"].hist_col.launches == 0
    # another workload's signature is not applied
    other = B.boruta_fit_ex(X[:1999], y[:1999], 3, 6, 8, stats=True,
                            tune=dict(tune_cache=cache), **kw)
    assert other["stats"].hist_col.launches == 0
    # the autotuner reads the same file back
    assert A.read_cache(cache)[sig] == dict(col_level=2, col_unit=7, hist_rb=4, hist_fw=1)
