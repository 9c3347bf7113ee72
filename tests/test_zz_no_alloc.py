"""The allocation-free entry point (boruta_fit_device_noalloc, for callers that
cannot allocate device memory) against boruta_fit_device with a caller
workspace: identical decisions, hits, history and shadow maxima, on two calls
in a row (the second smaller, so the scratch holds the first call's contents),
and a clear refusal of a problem larger than its scratch."""
import numpy as np
import pytest

from paper_2605_09950_amd import binding as B

pytestmark = pytest.mark.gpu


def problem(seed, n, p, K):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(np.float32)
    y = (np.argmax(X[:, :K] + 0.5 * rng.standard_normal((n, K)), axis=1)).astype(np.int32)
    return X, y


def same(a, b):
    assert a["n_iter"] == b["n_iter"]
    k = a["n_iter"]
    assert np.array_equal(a["decision"], b["decision"])
    assert np.array_equal(a["hits"], b["hits"])
    ha, hb = a["imp_history"][:k], b["imp_history"][:k]
    assert np.array_equal(np.isnan(ha), np.isnan(hb))
    assert np.array_equal(ha[~np.isnan(ha)], hb[~np.isnan(hb)])
    assert np.array_equal(a["shadow_max"][:k], b["shadow_max"][:k])


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    import torch
    cases = [  # second call smaller than the first
        dict(seed=61, n=3000, p=120, K=3, T=60, D=10, mode=B.PERMUT, iters=12),
        dict(seed=62, n=700, p=25, K=2, T=30, D=7, mode=B.TREEIMP, iters=15),
    ]
    for c in cases:
        print(f"no-alloc case n={c['n']} p={c['p']} mode={c['mode']}", flush=True)
        X, y = problem(c["seed"], c["n"], c["p"], c["K"])
        dX, dy = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        kw = dict(importance_mode=c["mode"], max_iter=c["iters"], seed=c["seed"] + 100)
        got = B.boruta_fit_device_noalloc(dX, dy, c["K"], c["T"], c["D"], **kw)
        shape = dict(n=c["n"], p=c["p"], n_classes=c["K"], n_trees=c["T"], max_depth=c["D"],
                     importance_mode=c["mode"], max_iter=c["iters"])
        ws = torch.empty(B.boruta_workspace_size([shape]), dtype=torch.uint8, device="cuda")
        want = B.boruta_fit_device(dX, dy, c["K"], c["T"], c["D"], ws, **kw)
        same(got, want)
        assert (got["decision"] != 0).any()


def test_noalloc_refuses_a_problem_beyond_its_scratch():
    import torch
    X, y = problem(63, 10000, 500, 3)  # about 380 MiB of workspace
    dX, dy = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    with pytest.raises(B.BorutaError) as e:
        B.boruta_fit_device_noalloc(dX, dy, 3, 200, 12, max_iter=100)
    assert e.value.code == B.BORUTA_E_INVALID_ARG
    assert "scratch" in B.boruta_last_error()
