"""Seeded synthetic workloads shaped like the paper's high-dimensional inputs.

The paper's datasets (its synthetic regression set, CT, NEWS, ENERGY and
MADELON, Sec. 3) are not available here, so every workload is generated from
a fixed seed.  This module only draws inputs (feature matrix, labels, run
parameters); it holds none of the selection method's arithmetic and is shared
by the HIP path's tests/benchmark and by the CPU oracle's tests.

Workloads (data seed / Boruta seed):
  0  planted check          n=500,    p=20,     K=2, 64 bins, 50 trees depth 8, 20 iterations
  1  MADELON-like           n=10000,  p=500,    K=3, 200 trees depth 12, 100 iterations
  2  omics-shaped           n=2000,   p=20000,  K=2, 500 trees depth 12, 100 iterations
  3  many small jobs        64 jobs, n in [200,5000], p in [50,2000], K in [2,5]
  4  precision + scale      n=100000, p=2000,   K=4, 300 trees depth 16, 100 iterations
  5  regression             n=10000,  p=50 U(0,1), 10 informative, float target,
                            200 trees depth 12, 100 iterations (the shape of the
                            paper's synthetic regression set; our own function)
"""
import numpy as np

TREEIMP, PERMUT = 0, 1


def _params(**kw):
    base = dict(n_bins=256, mtry=0, alpha=0.05, n_perm=1, importance_mode=TREEIMP)
    base.update(kw)
    return base


def planted_small(seed=1000, n=500, p=20, n_inf=5):
    """Binary label = sign(+-1 weighted sum of 5 informative N(0,1) columns
    plus N(0, sd 0.5) noise)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(np.float32)
    inf = np.sort(rng.choice(p, n_inf, replace=False))
    w = rng.choice([-1.0, 1.0], n_inf)
    score = X[:, inf].astype(np.float64) @ w + rng.normal(0.0, 0.5, n)
    y = (score > 0).astype(np.int32)
    return X, y, inf


def madelon_like(seed=1001, n=10000, n_inf=20, n_mix=80, n_noise=400, n_classes=3):
    """3-class label from the argmax of 3 random quadratic forms over 20
    informative columns, 80 noisy linear mixes of them, 400 N(0,1) noise
    columns, columns shuffled."""
    rng = np.random.default_rng(seed)
    XI = rng.standard_normal((n, n_inf))
    A = rng.standard_normal((n_classes, n_inf, n_inf)) / np.sqrt(n_inf)
    A = 0.5 * (A + A.transpose(0, 2, 1))
    scores = np.einsum("ni,cij,nj->nc", XI, A, XI)
    y = np.argmax(scores, axis=1).astype(np.int32)
    M = rng.standard_normal((n_inf, n_mix)) / np.sqrt(n_inf)
    mixes = XI @ M + rng.normal(0.0, 0.1, (n, n_mix))
    noise = rng.standard_normal((n, n_noise))
    full = np.concatenate([XI, mixes, noise], axis=1)
    order = rng.permutation(full.shape[1])
    X = np.ascontiguousarray(full[:, order], dtype=np.float32)
    inv = np.argsort(order)
    inf = np.sort(inv[:n_inf])
    mix_cols = np.sort(inv[n_inf:n_inf + n_mix])
    return X, y, inf, mix_cols


def omics_like(seed=1002, n=2000, p=20000, n_inf=50, flip=0.10):
    """Log-normal features, logistic binary label over 50 informative
    log-features, 10% of labels flipped."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, p)).astype(np.float32)
    inf = np.sort(rng.choice(p, n_inf, replace=False))
    beta = rng.standard_normal(n_inf) * (2.0 / np.sqrt(n_inf))
    logit = Z[:, inf].astype(np.float64) @ beta
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-logit))).astype(np.int32)
    flip_rows = rng.random(n) < flip
    y[flip_rows] = 1 - y[flip_rows]
    X = np.exp(Z).astype(np.float32)
    return X, y, inf


def many_job(j):
    """Job j of the 64-job batch: N(0,1) features, K-class argmax label over a
    5% informative subset."""
    rng = np.random.default_rng(4000 + j)
    n = int(rng.integers(200, 5001))
    p = int(rng.integers(50, 2001))
    K = int(rng.integers(2, 6))
    n_inf = max(1, int(round(0.05 * p)))
    X = rng.standard_normal((n, p)).astype(np.float32)
    inf = np.sort(rng.choice(p, n_inf, replace=False))
    W = rng.standard_normal((K, n_inf))
    scores = X[:, inf].astype(np.float64) @ W.T + rng.normal(0.0, 0.5, (n, K))
    y = np.argmax(scores, axis=1).astype(np.int32)
    return X, y, K, inf


def mixed_scale(seed=1004, n=100000, p=2000, n_inf=40, n_classes=4, depth=6):
    """45% N(0,1), 45% U(0,1) and 10% categorical-coded columns (2..16
    levels); 4-class label from a random depth-6 tree over 40 informative
    columns with thresholds at random U(0.2, 0.8) quantiles."""
    rng = np.random.default_rng(seed)
    kinds = rng.permutation(np.array([0] * int(0.45 * p) + [1] * int(0.45 * p) +
                                     [2] * (p - 2 * int(0.45 * p))))
    X = np.empty((n, p), dtype=np.float32)
    for j in range(p):
        if kinds[j] == 0:
            X[:, j] = rng.standard_normal(n)
        elif kinds[j] == 1:
            X[:, j] = rng.random(n)
        else:
            X[:, j] = rng.integers(0, int(rng.integers(2, 17)), n)
    # informative columns spread over the three kinds in proportion
    inf = np.sort(rng.choice(p, n_inf, replace=False))
    n_internal = 2 ** depth - 1
    feat = rng.choice(inf, n_internal)
    thr = np.array([np.quantile(X[:, f], rng.uniform(0.2, 0.8)) for f in feat])
    while True:
        leaf_cls = rng.integers(0, n_classes, 2 ** depth)
        if len(np.unique(leaf_cls)) == n_classes:
            break
    node = np.zeros(n, dtype=np.int64)  # 0-based heap index
    rows = np.arange(n)
    for _ in range(depth):
        go_left = X[rows, feat[node]] <= thr[node]
        node = 2 * node + 1 + (~go_left)
    y = leaf_cls[node - n_internal].astype(np.int32)
    return X, y, inf


def regression_like(seed=1005, n=10000, p=50, n_inf=10):
    """Float target over 10 of 50 U(0,1) columns: linear, sine, product,
    threshold and quadratic terms, plus N(0, sd 0.5) noise."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, p)).astype(np.float32)
    inf = np.sort(rng.choice(p, n_inf, replace=False))
    Z = X[:, inf].astype(np.float64)
    y = (5.0 * Z[:, 0] + 3.0 * np.sin(np.pi * Z[:, 1] * Z[:, 2]) + 4.0 * (Z[:, 3] - 0.5) ** 2
         + 2.0 * (Z[:, 4] > 0.5) + 1.5 * Z[:, 5] * Z[:, 6] + Z[:, 7] - Z[:, 8]
         + 0.5 * np.cos(2 * np.pi * Z[:, 9]) + rng.normal(0.0, 0.5, n))
    return X, y.astype(np.float32), inf


def config(i):
    """Workload i as a dict: X, y, informative columns and the run parameters."""
    if i == 0:
        X, y, inf = planted_small()
        return dict(X=X, y=y, informative=inf, n_classes=2, seed=7000,
                    params=_params(n_bins=64, n_trees=50, max_depth=8, max_iter=20))
    if i == 1:
        X, y, inf, mix = madelon_like()
        return dict(X=X, y=y, informative=inf, mixes=mix, n_classes=3, seed=7001,
                    params=_params(n_trees=200, max_depth=12, max_iter=100))
    if i == 2:
        X, y, inf = omics_like()
        return dict(X=X, y=y, informative=inf, n_classes=2, seed=7002,
                    params=_params(n_trees=500, max_depth=12, max_iter=100))
    if i == 4:
        X, y, inf = mixed_scale()
        return dict(X=X, y=y, informative=inf, n_classes=4, seed=7004,
                    params=_params(n_trees=300, max_depth=16, max_iter=100, n_perm=5))
    if i == 5:
        X, y, inf = regression_like()
        return dict(X=X, y_reg=y, informative=inf, seed=7005,
                    params=_params(n_trees=200, max_depth=12, max_iter=100))
    raise ValueError("workload 3 is a batch: use many_jobs()")


def many_jobs(n_jobs=64):
    jobs = []
    for j in range(n_jobs):
        X, y, K, inf = many_job(j)
        jobs.append(dict(X=X, y=y, informative=inf, n_classes=K, seed=8000 + j,
                         params=_params(n_trees=100, max_depth=10, max_iter=50,
                                        importance_mode=PERMUT)))
    return jobs
