"""Writes the stored oracle results of the whole-run parity tests: per
iteration, the digest of the CPU oracle's trace record (tree tables of every
tree, integer importances, hits, states; see tests/trace_digest.py), and per
run the final decisions, hits, rank and history digest.  Calls only the
oracle and the seeded input generators.

    python tests/golden/make_wholerun_golden.py PART... [--threads N]

Parts (each writes tests/golden/<part>.json):
  wholerun_madelon   MADELON-like n=10,000, p=500: whole runs (up to 100
                     iterations), TreeImp and Permut (one replica)
  wholerun_manyjob   the 64-job batch: every job's whole run (up to 50
                     iterations, Permut)
  iter1_omics        omics-shaped n=2,000, p=20,000: iteration 1, all 500 trees
  iter1_scale        mixed-type n=100,000, p=2,000: iteration 1, all 300 trees,
                     TreeImp and Permut with five replicas
  wholerun_omics     omics-shaped n=2,000, p=20,000: the whole TreeImp run
  iters4_scale       mixed-type n=100,000, p=2,000: TreeImp iterations 1..4
                     (a run stopped at max_iter = 4)
  wholerun_scale     mixed-type n=100,000, p=2,000: the whole TreeImp run
  wholerun_omics_permut   omics-shaped: the whole Permut run (one replica)
  wholerun_scale_permut   mixed-type: the whole Permut run (five replicas)
  wholerun_madelon_kl     MADELON-like: the whole Permut-KL run (Algorithm 3)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2605_09950_amd import synth  # noqa: E402
from tests.trace_digest import Digester, run_summary  # noqa: E402


def whole_run(X, y, K, pr, seed, mode, threads):
    dg = Digester()
    r = O.boruta_fit(X, y, K, pr["n_trees"], pr["max_depth"], mtry=pr["mtry"],
                     importance_mode=mode, max_iter=pr["max_iter"], alpha=pr["alpha"],
                     seed=seed, n_bins=pr["n_bins"], n_perm=pr["n_perm"], n_threads=threads,
                     trace=dg)
    return dict(run_summary(r), iterations=dg.by_job.get(0, []))


def first_iteration(c, mode, n_perm, threads):
    pr = c["params"]
    p = c["X"].shape[1]
    dg = Digester()
    r = O.boruta_step(c["X"], c["y"], c["n_classes"], pr["n_trees"], pr["max_depth"], 1,
                      np.zeros(p, np.int8), np.zeros(p, np.int32), mtry=pr["mtry"],
                      importance_mode=mode, alpha=pr["alpha"], seed=c["seed"],
                      n_bins=pr["n_bins"], n_perm=n_perm, n_threads=threads, trace=dg)
    return {"mode": mode, "n_perm": n_perm, "t": 1, "iterations": dg.by_job[0],
            "hits": np.asarray(r["hits"], np.int64).tolist(),
            "state": np.asarray(r["state"], np.int64).tolist()}


def part(name, threads):
    t0 = time.time()
    if name == "wholerun_madelon":
        c = synth.config(1)
        out = {"workload": "MADELON-like n=10000 p=500 K=3, 256 bins, 200 trees depth 12",
               "seed": c["seed"], "runs": {}}
        for mode in (0, 1):
            out["runs"][str(mode)] = whole_run(c["X"], c["y"], c["n_classes"], c["params"],
                                               c["seed"], mode, threads)
            print(name, "mode", mode, "iterations", out["runs"][str(mode)]["n_iter"],
                  f"{time.time() - t0:.0f}s", flush=True)
    elif name == "wholerun_manyjob":
        out = {"workload": "64 jobs, n in [200,5000], p in [50,2000], K in [2,5], 100 trees "
                           "depth 10, Permut", "jobs": []}
        for j, c in enumerate(synth.many_jobs()):
            pr = c["params"]
            out["jobs"].append(whole_run(c["X"], c["y"], c["n_classes"], pr, c["seed"],
                                         pr["importance_mode"], threads))
            print(name, "job", j, "iterations", out["jobs"][-1]["n_iter"],
                  f"{time.time() - t0:.0f}s", flush=True)
    elif name == "iter1_omics":
        c = synth.config(2)
        out = {"workload": "omics-shaped n=2000 p=20000 K=2, 256 bins, 500 trees depth 12",
               "seed": c["seed"], "legs": [first_iteration(c, 0, 1, threads)]}
    elif name == "iter1_scale":
        c = synth.config(4)
        out = {"workload": "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16",
               "seed": c["seed"], "legs": []}
        for mode, n_perm in ((0, 1), (1, 5)):
            out["legs"].append(first_iteration(c, mode, n_perm, threads))
            print(name, "mode", mode, f"{time.time() - t0:.0f}s", flush=True)
    elif name == "wholerun_omics":
        c = synth.config(2)
        out = {"workload": "omics-shaped n=2000 p=20000 K=2, 256 bins, 500 trees depth 12",
               "seed": c["seed"],
               "runs": {"0": whole_run(c["X"], c["y"], c["n_classes"], c["params"], c["seed"],
                                       0, threads)}}
    elif name == "iters4_scale":
        c = synth.config(4)
        pr = dict(c["params"], max_iter=4)
        out = {"workload": "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16",
               "seed": c["seed"], "max_iter": 4,
               "runs": {"0": whole_run(c["X"], c["y"], c["n_classes"], pr, c["seed"], 0,
                                       threads)}}
    elif name == "wholerun_scale":
        c = synth.config(4)
        out = {"workload": "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16",
               "seed": c["seed"],
               "runs": {"0": whole_run(c["X"], c["y"], c["n_classes"], c["params"], c["seed"],
                                       0, threads)}}
    elif name in ("wholerun_omics_permut", "wholerun_scale_permut"):
        c = synth.config(2 if "omics" in name else 4)
        out = {"workload": ("omics-shaped n=2000 p=20000 K=2, 256 bins, 500 trees depth 12"
                            if "omics" in name else
                            "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16"),
               "seed": c["seed"], "n_perm": c["params"]["n_perm"],
               "runs": {"1": whole_run(c["X"], c["y"], c["n_classes"], c["params"], c["seed"],
                                       1, threads)}}
    elif name == "wholerun_madelon_kl":
        c = synth.config(1)
        out = {"workload": "MADELON-like n=10000 p=500 K=3, 256 bins, 200 trees depth 12",
               "seed": c["seed"],
               "runs": {"2": whole_run(c["X"], c["y"], c["n_classes"], c["params"], c["seed"],
                                       2, threads)}}
    else:
        raise SystemExit(f"unknown part {name}")
    out["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)
    print(name, "written", f"{time.time() - t0:.0f}s", flush=True)


def main():
    args = sys.argv[1:]
    threads = 0
    if "--threads" in args:
        i = args.index("--threads")
        threads = int(args[i + 1])
        del args[i:i + 2]
    for name in args:
        part(name, threads)


if __name__ == "__main__":
    main()
