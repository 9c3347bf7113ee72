"""Writes fullsize_trees.json: for sampled trees of the first iteration of
the omics-shaped (n=2000, p=20000) and mixed-type (n=100000, p=2000)
workloads, the CPU oracle's node table (SHA-256 of the int64 rows
[tree, heap, feature, threshold or leaf class, N, gain]) and per-tree
statistics.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_fullsize_golden.py [n_threads]
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2605_09950_amd import synth  # noqa: E402

SAMPLES = {2: [0, 1, 250, 499], 4: [0, 150]}


def node_digest(nodes):
    a = np.ascontiguousarray(nodes, dtype=np.int64)
    return hashlib.sha256(a.tobytes()).hexdigest()


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    out = {}
    for i, trees in SAMPLES.items():
        c = synth.config(i)
        pr = c["params"]
        p = c["X"].shape[1]
        r = O.boruta_step(c["X"], c["y"], c["n_classes"], pr["n_trees"], pr["max_depth"], 1,
                          np.zeros(p, np.int8), np.zeros(p, np.int32), mtry=pr["mtry"],
                          importance_mode=0, alpha=pr["alpha"], seed=c["seed"],
                          n_bins=pr["n_bins"], n_perm=pr["n_perm"], tree_subset=trees,
                          n_threads=threads, trace=True)
        tr = r["trace"]
        out[str(i)] = {"trees": trees, "t": 1, "p_w": int(tr["p_w"]), "mtry": int(tr["mtry"]),
                       "n_nodes": int(tr["nodes"].shape[0]),
                       "nodes_sha256": node_digest(tr["nodes"]),
                       "tree_stats": np.asarray(tr["tree_stats"], dtype=np.int64).tolist()}
        print(i, out[str(i)]["n_nodes"], out[str(i)]["nodes_sha256"][:16], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_trees.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
