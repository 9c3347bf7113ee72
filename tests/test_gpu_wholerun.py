"""Whole Boruta runs of the HIP path against stored oracle results
(tests/golden/*.json, written by tests/golden/make_wholerun_golden.py, which
calls only the oracle): per iteration the digest of the trace record (every
tree's node table, integer importances, hits, states, per-tree statistics)
and per run the decisions, hits, rank and history.  Launch configuration of
bench.py: a session over device-resident inputs and a caller workspace,
iterations replayed from the captured graph.

  * MADELON-like n=10,000, p=500: whole runs in TreeImp and Permut, FP32 and
    exact-only ranking, and in Permut-KL;
  * the 64-job batch: every job's whole run, all jobs in one session;
  * omics-shaped n=2,000, p=20,000 and mixed-type n=100,000, p=2,000: the
    whole first iteration (every tree), both ranking modes; mixed-type also
    with Permut and five replicas;
  * omics-shaped and mixed-type: the whole TreeImp run (mixed-type also its
    iterations 1-4 as a run stopped at max_iter = 4) and the whole Permut run
    (one replica for the omics shape, five for mixed-type).
"""
import json
import os

import numpy as np
import pytest

from paper_2605_09950_amd import binding as B
from paper_2605_09950_amd import synth
from tests.trace_digest import Digester, run_summary

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLD, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    with open(path) as f:
        return json.load(f)


def run_session(jobs, n_bins, n_perm=1, rank=B.RANK_FP32, steps=None, tune=None):
    """A session shaped like the bench's; every iteration's record digested.
    Returns (digests per job, results per job)."""
    import torch
    dev = []
    for jd in jobs:
        d = dict(jd)
        d["X"] = torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda()
        d["y"] = torch.from_numpy(np.ascontiguousarray(jd["y"])).cuda()
        dev.append(d)
    shapes = [dict(n=d["X"].shape[0], p=d["X"].shape[1],
                   **{k: v for k, v in d.items() if k not in ("X", "y")}) for d in dev]
    ws = torch.empty(B.boruta_workspace_size(shapes, n_bins=n_bins, n_perm=n_perm,
                                             split_rank=rank, tune=tune),
                     dtype=torch.uint8, device="cuda")
    dg = Digester()
    with B.Session(dev, n_bins=n_bins, n_perm=n_perm, split_rank=rank, trace=dg,
                   inputs_on_device=True, workspace=ws, stream=torch.cuda.current_stream(),
                   graph=True, tune=tune) as s:
        live, k = len(jobs), 0
        while live and (steps is None or k < steps):
            live = s.step()
            k += 1
        res = [s.result(j) for j in range(len(jobs))]
    torch.cuda.synchronize()
    return dg.by_job, res


def compare_iterations(got, want, what):
    for i, (g, w) in enumerate(zip(got, want)):
        assert g["digest"] == w["digest"], (
            f"{what}: first differing iteration {w['t']}: gpu {g} oracle {w}")
    assert len(got) == len(want), (what, len(got), len(want))


def compare_run(res, want, what):
    got = run_summary(res)
    for k in ("n_iter", "decision", "hits", "rank", "history_sha256", "shadow_max_sha256"):
        assert got[k] == want[k], (what, k)


def job(c, mode):
    pr = c["params"]
    return dict(X=c["X"], y=c["y"], n_classes=c["n_classes"], n_trees=pr["n_trees"],
                max_depth=pr["max_depth"], mtry=pr["mtry"], importance_mode=mode,
                max_iter=pr["max_iter"], alpha=pr["alpha"], seed=c["seed"])


@pytest.mark.parametrize("mode,rank", [(0, B.RANK_FP32), (1, B.RANK_FP32), (0, B.RANK_EXACT)])
def test_madelon_whole_run(mode, rank):
    g = golden("wholerun_madelon")
    want = g["runs"][str(mode)]
    c = synth.config(1)
    print(f"madelon whole run mode {mode} rank {rank}", flush=True)
    dig, res = run_session([job(c, mode)], c["params"]["n_bins"], rank=rank)
    compare_iterations(dig[0], want["iterations"], f"madelon mode {mode}")
    compare_run(res[0], want, f"madelon mode {mode}")


def test_madelon_whole_run_permut_kl():
    # the whole run with Algorithm 3's importance
    g = golden("wholerun_madelon_kl")
    want = g["runs"]["2"]
    c = synth.config(1)
    print("madelon whole run Permut-KL", flush=True)
    dig, res = run_session([job(c, 2)], c["params"]["n_bins"])
    compare_iterations(dig[0], want["iterations"], "madelon Permut-KL")
    compare_run(res[0], want, "madelon Permut-KL")


def test_madelon_whole_run_back_to_back():
    # the bench's whole-run form: iterations enqueued back to back, no trace
    import torch
    g = golden("wholerun_madelon")
    want = g["runs"]["0"]
    c = synth.config(1)
    jd = job(c, 0)
    d = dict(jd, X=torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda(),
             y=torch.from_numpy(np.ascontiguousarray(jd["y"])).cuda())
    shapes = [dict(n=d["X"].shape[0], p=d["X"].shape[1],
                   **{k: v for k, v in d.items() if k not in ("X", "y")})]
    ws = torch.empty(B.boruta_workspace_size(shapes, n_bins=256), dtype=torch.uint8,
                     device="cuda")
    with B.Session([d], n_bins=256, inputs_on_device=True, workspace=ws,
                   stream=torch.cuda.current_stream()) as s:
        s.run(jd["max_iter"])
        r = s.result(0)
    compare_run(r, want, "madelon back to back")


def test_strided_device_inputs_are_refused():
    # a device input is handed over as a raw pointer; a column-major view of X
    # would be read as row-major, so the binding refuses it
    import torch
    c = synth.config(0)
    X = torch.from_numpy(np.asfortranarray(c["X"])).cuda()
    assert not X.is_contiguous()
    d = dict(job(c, 0), X=X, y=torch.from_numpy(c["y"]).cuda())
    with pytest.raises(ValueError):
        B.Session([d], n_bins=64, inputs_on_device=True)


def test_manyjob_whole_runs():
    g = golden("wholerun_manyjob")
    cs = synth.many_jobs()
    jobs = [job(c, c["params"]["importance_mode"]) for c in cs]
    print("64-job batch whole runs", flush=True)
    dig, res = run_session(jobs, 256)
    for j, want in enumerate(g["jobs"]):
        compare_iterations(dig[j], want["iterations"], f"job {j}")
        compare_run(res[j], want, f"job {j}")


@pytest.mark.parametrize("rank", [B.RANK_FP32, B.RANK_EXACT])
def test_omics_first_iteration(rank):
    g = golden("iter1_omics")
    c = synth.config(2)
    leg = g["legs"][0]
    print(f"omics iteration 1 rank {rank}", flush=True)
    dig, res = run_session([job(c, leg["mode"])], 256, n_perm=leg["n_perm"], rank=rank, steps=1)
    compare_iterations(dig[0], leg["iterations"], "omics iteration 1")
    assert res[0]["hits"].tolist() == leg["hits"]


@pytest.mark.parametrize("leg_i,rank", [(0, B.RANK_FP32), (0, B.RANK_EXACT), (1, B.RANK_FP32)])
def test_scale_first_iteration(leg_i, rank):
    g = golden("iter1_scale")
    c = synth.config(4)
    leg = g["legs"][leg_i]
    print(f"mixed-type iteration 1 mode {leg['mode']} rank {rank}", flush=True)
    dig, res = run_session([job(c, leg["mode"])], 256, n_perm=leg["n_perm"], rank=rank, steps=1)
    compare_iterations(dig[0], leg["iterations"], f"mixed-type iteration 1 mode {leg['mode']}")
    assert res[0]["hits"].tolist() == leg["hits"]


@pytest.mark.parametrize("rank", [B.RANK_FP32, B.RANK_EXACT])
def test_omics_whole_run(rank):
    g = golden("wholerun_omics")
    want = g["runs"]["0"]
    c = synth.config(2)
    print(f"omics whole run rank {rank}", flush=True)
    dig, res = run_session([job(c, 0)], c["params"]["n_bins"], rank=rank)
    compare_iterations(dig[0], want["iterations"], "omics whole run")
    compare_run(res[0], want, "omics whole run")


@pytest.mark.parametrize("rank", [B.RANK_FP32, B.RANK_EXACT])
def test_scale_first_four_iterations(rank):
    # a run stopped at max_iter = 4: decisions, hits, rank and history of the
    # truncated run, and every iteration's trace digest
    g = golden("iters4_scale")
    want = g["runs"]["0"]
    c = synth.config(4)
    jd = dict(job(c, 0), max_iter=g["max_iter"])
    print(f"mixed-type iterations 1-4 rank {rank}", flush=True)
    dig, res = run_session([jd], c["params"]["n_bins"], rank=rank)
    compare_iterations(dig[0], want["iterations"], "mixed-type iterations 1-4")
    compare_run(res[0], want, "mixed-type iterations 1-4")


@pytest.mark.parametrize("rank", [B.RANK_FP32, B.RANK_EXACT])
def test_scale_whole_run(rank):
    g = golden("wholerun_scale")
    want = g["runs"]["0"]
    c = synth.config(4)
    print(f"mixed-type whole run rank {rank}", flush=True)
    dig, res = run_session([job(c, 0)], c["params"]["n_bins"], rank=rank)
    compare_iterations(dig[0], want["iterations"], "mixed-type whole run")
    compare_run(res[0], want, "mixed-type whole run")


@pytest.mark.parametrize("name,cfg", [("wholerun_omics_permut", 2),
                                      ("wholerun_scale_permut", 4)])
def test_permut_whole_run(name, cfg):
    # the whole Permut run with the workload's own replica count (one for the
    # omics shape, five for mixed-type)
    g = golden(name)
    want = g["runs"]["1"]
    c = synth.config(cfg)
    assert g["n_perm"] == c["params"]["n_perm"]
    print(f"{name}: whole Permut run, {g['n_perm']} replicas", flush=True)
    dig, res = run_session([job(c, 1)], c["params"]["n_bins"], n_perm=g["n_perm"])
    compare_iterations(dig[0], want["iterations"], name)
    compare_run(res[0], want, name)
