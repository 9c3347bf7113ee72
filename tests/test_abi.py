"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/boruta.h declares, validates arguments on the host, sizes workspaces,
and fails loudly (no CPU fallback) when no GPU is present."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_09950_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "boruta.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(boruta_[a-z_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_binding_exports():
    assert header_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_default_options():
    o = B.boruta_default_options()
    assert (o.n_bins, o.n_perm, o.split_rank, o.form) == (256, 1, B.RANK_FP32, B.FORM_BATCHED)
    assert (o.graph, o.small_rows, o.grid_small, o.grid_hist, o.grid_finalize) == (1, 32, 0, 0, 0)
    assert (o.col_level, o.col_unit, o.grid_col, o.kl_rows) == (0, 2048, 0, 0)
    assert (o.perc, o.rough_fix) == (100, 0)
    assert not o.trace and not o.stats


@pytest.mark.parametrize("field,value", [("perc", 101), ("perc", -1), ("rough_fix", 2)])
def test_percentile_and_rough_fix_validated_on_the_host(field, value):
    import ctypes
    o, _ = B.make_options()
    setattr(o, field, value)
    job = (B.Job * 1)()
    job[0].X = job[0].y = 1
    job[0].n, job[0].p, job[0].n_classes, job[0].n_trees = 100, 5, 2, 2
    job[0].max_depth, job[0].max_iter, job[0].alpha = 3, 3, 0.05
    out = ctypes.c_size_t(0)
    rc = B.lib().boruta_workspace_size(job, 1, ctypes.byref(o), ctypes.byref(out))
    assert rc == B.BORUTA_E_INVALID_ARG
    assert "perc" in B.boruta_last_error() or "rough_fix" in B.boruta_last_error()


def test_tuning_options_validated_on_the_host():
    for tune in (dict(small_rows=1), dict(small_rows=65), dict(grid_hist=-1),
                 dict(grid_small=70000), dict(col_level=-1), dict(col_level=65),
                 dict(col_unit=-2), dict(col_unit=65537), dict(grid_col=70000),
                 dict(kl_rows=-1)):
        with pytest.raises(B.BorutaError) as e:
            B.boruta_workspace_size([dict(n=100, p=5, n_classes=2, n_trees=2, max_depth=3)],
                                    tune=tune)
        assert e.value.code == B.BORUTA_E_INVALID_ARG
    with pytest.raises(ValueError):
        B.make_options(tune=dict(bogus=1))


def test_small_rows_sizes_the_large_node_lists():
    job = [dict(n=5000, p=50, n_classes=3, n_trees=10, max_depth=10)]
    assert B.boruta_workspace_size(job, tune=dict(small_rows=16)) > B.boruta_workspace_size(job)
    assert B.boruta_workspace_size(job, tune=dict(small_rows=64)) < B.boruta_workspace_size(job)


def test_column_path_buffers_only_when_a_level_uses_it():
    # depth 8: col_level 5 puts levels 5..7 on the column-major path; col_level
    # 64 (never) or a tree too shallow to reach col_level plans no column buffers
    job = [dict(n=5000, p=50, n_classes=3, n_trees=10, max_depth=8)]
    never = B.boruta_workspace_size(job, tune=dict(col_level=64))
    assert B.boruta_workspace_size(job, tune=dict(col_level=5)) > never
    assert B.boruta_workspace_size(job, tune=dict(col_level=8)) == never
    assert B.boruta_workspace_size(job, tune=dict(col_level=7)) > never
    # automatic choice: a 100 KB-column, 4000-column matrix (about 400 MB)
    # takes it, a small one does not
    assert B.boruta_workspace_size(job) == never
    big = [dict(n=100000, p=2000, n_classes=4, n_trees=2, max_depth=8)]
    assert (B.boruta_workspace_size(big) ==
            B.boruta_workspace_size(big, tune=dict(col_level=5)) >
            B.boruta_workspace_size(big, tune=dict(col_level=64)))
    # the plain form never takes it
    assert (B.boruta_workspace_size(job, form=B.FORM_PLAIN) ==
            B.boruta_workspace_size(job, form=B.FORM_PLAIN, tune=dict(col_level=64)))
    # a column wider than a workgroup's LDS (n = 200,000 rows) keeps every level
    # node-major
    wide = [dict(n=200000, p=4, n_classes=2, n_trees=1, max_depth=8)]
    assert (B.boruta_workspace_size(wide) ==
            B.boruta_workspace_size(wide, tune=dict(col_level=64)))


def test_kl_buffers_sized_by_row_block():
    job = [dict(n=5000, p=50, n_classes=3, n_trees=10, max_depth=8, importance_mode=2)]
    other = [dict(job[0], importance_mode=1)]
    full = B.boruta_workspace_size(job)
    # one block of all rows: differences [p_w][n][K] u64 plus the row sums
    assert full >= B.boruta_workspace_size(other) + 100 * 5000 * 3 * 8
    assert B.boruta_workspace_size(job, tune=dict(kl_rows=100)) < full
    assert B.boruta_workspace_size(job, tune=dict(kl_rows=100000)) == full


def _call(**kw):
    args = dict(X=np.zeros((10, 3), np.float32), y=np.zeros(10, np.int32), n_classes=2,
                n_trees=2, max_depth=2, max_iter=3)
    args.update(kw)
    return B.boruta_fit_ex(**args)


@pytest.mark.parametrize("kw", [dict(n_classes=1), dict(n_classes=17), dict(n_trees=0),
                                dict(max_depth=0), dict(max_depth=31), dict(max_iter=0),
                                dict(max_iter=1001), dict(alpha=0.5), dict(alpha=0.0),
                                dict(mtry=-1), dict(importance_mode=3), dict(importance_mode=-1), dict(n_bins=1),
                                dict(n_bins=257), dict(n_perm=0), dict(split_rank=2),
                                dict(form=3), dict(X=np.zeros((1, 3), np.float32),
                                                   y=np.zeros(1, np.int32))])
def test_invalid_arguments_rejected_on_host(kw):
    with pytest.raises(B.BorutaError) as e:
        _call(**kw)
    assert e.value.code == B.BORUTA_E_INVALID_ARG
    assert B.boruta_last_error()


@pytest.mark.parametrize("seeds", [[], list(range(65))], ids=["none", "65"])
def test_seed_count_rejected_on_host(seeds):
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_seeds(np.zeros((10, 3), np.float32), np.zeros(10, np.int32), 2, 2, 2,
                           seeds, max_iter=3)
    assert e.value.code == B.BORUTA_E_INVALID_ARG


def test_regression_arguments_checked_on_the_host():
    X = np.zeros((50, 2), np.float32)
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_regression(X, np.zeros(50, np.float32), 2, 2, importance_mode=3)
    assert e.value.code == B.BORUTA_E_INVALID_ARG
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_regression(X[:1], np.zeros(1, np.float32), 2, 2)
    assert e.value.code == B.BORUTA_E_INVALID_ARG
    # no row cap below 2^24 and no cap on n_trees * n * n_perm: past the host
    # checks, the call fails only for want of a device here
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_regression(np.zeros((70000, 2), np.float32), np.zeros(70000, np.float32),
                                40000, 2, importance_mode=B.PERMUT, max_iter=2)
    assert e.value.code == B.BORUTA_E_UNSUPPORTED


def test_workspace_size_is_host_only():
    small = B.boruta_workspace_size([dict(n=500, p=20, n_classes=2, n_trees=50, max_depth=8)])
    big = B.boruta_workspace_size([dict(n=10000, p=500, n_classes=3, n_trees=200,
                                        max_depth=12, max_iter=100)])
    assert 0 < small < big
    two = B.boruta_workspace_size([dict(n=500, p=20, n_classes=2, n_trees=50, max_depth=8)] * 2)
    assert two > small
    with pytest.raises(B.BorutaError):
        B.boruta_workspace_size([dict(n=1, p=20, n_classes=2, n_trees=50, max_depth=8)])


def test_no_cpu_fallback_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.BorutaError) as e:
        _call()
    assert e.value.code == B.BORUTA_E_UNSUPPORTED
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_seeds(np.zeros((10, 3), np.float32), np.zeros(10, np.int32), 2, 2, 2,
                           [1, 2], max_iter=3)
    assert e.value.code == B.BORUTA_E_UNSUPPORTED
