"""HIP path vs CPU oracle at the full workload sizes, in the launch
configuration bench.py times (a session over device-resident inputs, a
caller-provided workspace, iterations replayed from the captured graph).

  * MADELON-like (n=10,000, p=500, 200 trees of depth 12): the whole first
    iteration, every tree, both out-of-bag importance modes, against the
    oracle run live; with the divergence importance (Algorithm 3), every tree
    and 24 sampled columns' scores.
  * Many-job batch (64 jobs of uneven n, p and class count): the first
    iteration of sampled jobs, every tree, against the oracle run live.
  * Regression (n=10,000, p=50, 200 trees of depth 12): every tree of the
    first iteration in all three importance modes, against the oracle run
    live.
  * Omics-shaped (n=2,000, p=20,000) and mixed-type (n=100,000, p=2,000):
    sampled trees of the first iteration against the node-table digests in
    tests/golden/fullsize_trees.json (written by make_fullsize_golden.py,
    which calls only the oracle), plus the trees' in-bag / OOB counts.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_09950_amd import binding as B
from paper_2605_09950_amd import synth
from tests.parity_helpers import assert_same_trace

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_trees.json")


def gpu_first_iteration(jobs, n_bins, n_perm=1, tune=None):
    """One step of a session shaped like the bench's; returns the traces."""
    import torch
    dev = []
    for jd in jobs:
        d = dict(jd)
        d["X"] = torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda()
        for key in ("y", "y_reg"):
            if key in jd:
                d[key] = torch.from_numpy(np.ascontiguousarray(jd[key])).cuda()
        dev.append(d)
    shapes = [dict(n=d["X"].shape[0], p=d["X"].shape[1], regression="y_reg" in d,
                   **{k: v for k, v in d.items() if k not in ("X", "y", "y_reg")})
              for d in dev]
    ws_bytes = B.boruta_workspace_size(shapes, n_bins=n_bins, n_perm=n_perm, tune=tune)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    with B.Session(dev, n_bins=n_bins, n_perm=n_perm, trace={1}, inputs_on_device=True,
                   workspace=ws, stream=stream, graph=True, tune=tune) as s:
        s.step()
        traces = list(s.traces)
    torch.cuda.synchronize()
    return traces


def job_of(c, mode=None):
    pr = c["params"]
    return dict(X=c["X"], y=c["y"], n_classes=c["n_classes"], n_trees=pr["n_trees"],
                max_depth=pr["max_depth"], mtry=pr["mtry"],
                importance_mode=pr["importance_mode"] if mode is None else mode,
                max_iter=pr["max_iter"], alpha=pr["alpha"], seed=c["seed"])


def oracle_first_iteration(jd, n_bins, n_perm=1, trees=None, kl_cols=None):
    p = jd["X"].shape[1]
    return O.boruta_step(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"], jd["max_depth"], 1,
                         np.zeros(p, np.int8), np.zeros(p, np.int32), mtry=jd["mtry"],
                         importance_mode=jd["importance_mode"], alpha=jd["alpha"],
                         seed=jd["seed"], n_bins=n_bins, n_perm=n_perm, tree_subset=trees,
                         n_threads=min(16, os.cpu_count() or 1), trace=True, kl_cols=kl_cols)


# the automatic choice keeps these workloads node-major; the column-major path
# (col_level 5) is checked on them as well
@pytest.mark.parametrize("tune", [None, dict(col_level=5)], ids=["auto", "column"])
@pytest.mark.parametrize("mode", [B.TREEIMP, B.PERMUT])
def test_madelon_like_first_iteration_all_trees(mode, tune):
    c = synth.config(1)
    pr = c["params"]
    jd = job_of(c, mode)
    print(f"MADELON-like n=10000 p=500 T=200 D=12 mode={mode} tune={tune}", flush=True)
    g = gpu_first_iteration([jd], pr["n_bins"], pr["n_perm"], tune=tune)
    assert len(g) == 1 and g[0]["t"] == 1
    o = oracle_first_iteration(jd, pr["n_bins"], pr["n_perm"])
    assert_same_trace(g[0], o["trace"])
    assert np.array_equal(g[0]["hits"], o["hits"])
    assert np.array_equal(g[0]["state"], o["state"])


def test_madelon_like_kl_sampled_columns():
    # Algorithm 3 at full size: every tree of the first iteration, and the
    # divergence scores of 24 sampled widened columns (originals and shadows)
    c = synth.config(1)
    pr = c["params"]
    jd = job_of(c, B.PERMUT_KL)
    print("MADELON-like n=10000 p=500 T=200 D=12 mode=KL, 24 sampled columns", flush=True)
    g = gpu_first_iteration([jd], pr["n_bins"])[0]
    cols = sorted(set(np.linspace(0, g["p_w"] - 1, 24).astype(int).tolist()))
    o = oracle_first_iteration(jd, pr["n_bins"], kl_cols=cols)["trace"]
    assert np.array_equal(g["nodes"], o["nodes"])
    assert np.array_equal(g["tree_stats"], o["tree_stats"])
    assert np.array_equal(g["imp_int"][cols], o["imp_int"][cols])
    assert (g["imp_int"][cols] > 0).sum() >= 4  # used columns carry nonzero scores


@pytest.mark.parametrize("tune", [None, dict(col_level=5)], ids=["auto", "column"])
def test_many_job_batch_sampled_jobs(tune):
    jobs = [dict(X=j["X"], y=j["y"], n_classes=j["n_classes"],
                 n_trees=j["params"]["n_trees"], max_depth=j["params"]["max_depth"],
                 mtry=j["params"]["mtry"], importance_mode=j["params"]["importance_mode"],
                 max_iter=j["params"]["max_iter"], alpha=j["params"]["alpha"], seed=j["seed"])
            for j in synth.many_jobs()]
    print(f"many-job batch: 64 jobs, sampled 0, 17, 40, 63, tune={tune}", flush=True)
    g = gpu_first_iteration(jobs, 256, tune=tune)
    by_job = {t["job"]: t for t in g}
    assert sorted(by_job) == list(range(64))
    for j in (0, 17, 40, 63):
        o = oracle_first_iteration(jobs[j], 256)
        assert_same_trace(by_job[j], o["trace"])
        assert np.array_equal(by_job[j]["hits"], o["hits"])
        assert np.array_equal(by_job[j]["state"], o["state"])


@pytest.mark.parametrize("mode", [B.TREEIMP, B.PERMUT, B.PERMUT_KL])
def test_regression_first_iteration_all_trees(mode):
    c = synth.config(5)
    pr = c["params"]
    jd = dict(X=c["X"], y_reg=c["y_reg"], n_trees=pr["n_trees"], max_depth=pr["max_depth"],
              mtry=pr["mtry"], importance_mode=mode, max_iter=pr["max_iter"], alpha=pr["alpha"],
              seed=c["seed"])
    print(f"regression n=10000 p=50 T=200 D=12 mode={mode}", flush=True)
    g = gpu_first_iteration([jd], pr["n_bins"])
    assert len(g) == 1 and g[0]["t"] == 1
    o = O.boruta_fit_reg(c["X"], c["y_reg"], pr["n_trees"], pr["max_depth"], mtry=pr["mtry"],
                         importance_mode=mode, max_iter=1, alpha=pr["alpha"], seed=c["seed"],
                         n_bins=pr["n_bins"], n_threads=min(16, os.cpu_count() or 1),
                         trace=True)
    assert_same_trace(g[0], o["traces"][0])
    assert np.array_equal(g[0]["hits"], o["hits"])
    assert np.array_equal(g[0]["state"], o["decision"])


def digest(nodes):
    return hashlib.sha256(np.ascontiguousarray(nodes, dtype=np.int64).tobytes()).hexdigest()


# omics: node-major by the automatic choice, also run on the column-major path;
# mixed (a 400 MB widened matrix): column-major from level 5 automatically,
# also run node-major
@pytest.mark.parametrize("tune", [None, "other"], ids=["auto", "other_path"])
@pytest.mark.parametrize("idx", [2, 4], ids=["omics_n2000_p20000", "mixed_n100000_p2000"])
def test_sampled_trees_match_oracle_digests(idx, tune):
    if tune == "other":
        tune = dict(col_level=5) if idx == 2 else dict(col_level=64)
    with open(GOLDEN) as f:
        ref = json.load(f)[str(idx)]
    c = synth.config(idx)
    pr = c["params"]
    jd = job_of(c, B.TREEIMP)
    print(f"workload {idx}: n={c['X'].shape[0]} p={c['X'].shape[1]} T={pr['n_trees']} "
          f"D={pr['max_depth']}, trees {ref['trees']}", flush=True)
    g = gpu_first_iteration([jd], pr["n_bins"], tune=tune)[0]
    assert (g["t"], g["p_w"], g["mtry"]) == (ref["t"], ref["p_w"], ref["mtry"])
    nodes = g["nodes"][np.isin(g["nodes"][:, 0], ref["trees"])]
    assert nodes.shape[0] == ref["n_nodes"]
    assert digest(nodes) == ref["nodes_sha256"]
    stats = g["tree_stats"][np.isin(g["tree_stats"][:, 0], ref["trees"])]
    assert np.array_equal(stats, np.asarray(ref["tree_stats"], dtype=np.int64))
