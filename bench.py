"""Benchmark: Boruta iterations/s on one MI355X, with the histogram kernel's
algorithmic bandwidth against the HBM roofline and the CPU oracle beside it.

A step is one Boruta iteration (shadow widening, bootstrap, random forest,
importance, hits, decision) of the MADELON-like workload: n=10,000 rows,
p=500 float32 features (20 informative, 80 noisy mixes, 400 noise), 3
classes, 256 quantile bins, 200 trees of depth 12, mtry = floor(sqrt(p_w)).
Inputs are resident in device memory (torch tensors) before the timed
region; binning happens once per job, at session creation, outside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Boruta iters/s + histogram HBM GB/s vs peak; batched/FP32 vs plain, exact"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["treeimp", "permut"], default="treeimp")
    ap.add_argument("--workload", choices=["madelon", "planted", "omics", "scale"],
                    default="madelon")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the Permut / exact / plain comparison legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="BYTES",
                    help="only run the library's streaming copy kernel over BYTES bytes "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def probe_copy(nbytes):
    """Five launches of the library's 16-byte-per-lane streaming copy."""
    import torch
    from paper_2605_09950_amd import binding as B
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        B.boruta_probe_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    assert bool((dst == 1).all())
    print(json.dumps({"probe_copy_bytes": nbytes, "launches": 5}), flush=True)


def workload(name):
    from paper_2605_09950_amd import synth
    idx = {"planted": 0, "madelon": 1, "omics": 2, "scale": 4}[name]
    c = synth.config(idx)
    pr = c["params"]
    n, p = c["X"].shape
    desc = {
        "planted": "planted n=500 p=20 K=2, 64 bins, 50 trees depth 8",
        "madelon": "MADELON-like n=10000 p=500 K=3 (20 informative, 80 mixes), 256 bins, "
                   "200 trees depth 12",
        "omics": "omics-shaped n=2000 p=20000 K=2 log-normal, 256 bins, 500 trees depth 12",
        "scale": "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16",
    }[name]
    return c, pr, n, p, desc


def run_gpu(c, pr, mode, steps, warmup, form, rank, stats, graph=True):
    import torch
    from paper_2605_09950_amd import binding as B
    dX = torch.from_numpy(c["X"]).cuda()
    dy = torch.from_numpy(c["y"]).cuda()
    job = dict(X=dX, y=dy, n_classes=c["n_classes"], n_trees=pr["n_trees"],
               max_depth=pr["max_depth"], mtry=pr["mtry"], importance_mode=mode,
               max_iter=min(1000, warmup + steps), alpha=pr["alpha"], seed=c["seed"])
    shape = dict(n=dX.shape[0], p=dX.shape[1], **{k: v for k, v in job.items()
                                                   if k not in ("X", "y")})
    ws_bytes = B.boruta_workspace_size([shape], n_bins=pr["n_bins"], n_perm=pr["n_perm"])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sess = B.Session([job], n_bins=pr["n_bins"], n_perm=pr["n_perm"], split_rank=rank,
                     form=form, stats=stats, inputs_on_device=True, workspace=ws,
                     stream=stream, graph=graph)
    for _ in range(warmup):
        sess.step()
    torch.cuda.synchronize()
    if sess.stats is not None:  # count only the timed iterations
        for f in ("hist_large", "hist_small", "finalize", "permut"):
            k = getattr(sess.stats, f)
            k.launches, k.ms, k.alg_bytes = 0, 0.0, 0.0
        sess.stats.iter_ms, sess.stats.iterations, sess.stats.nodes = 0.0, 0, 0
        for d in range(32):
            sess.stats.level_small[d] = sess.stats.level_large[d] = 0
    done = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        live = sess.step()
        done += 1
        if live == 0:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = sess.result(0)
    out = dict(steps=done, seconds=el, n_iter=res["n_iter"], stats=sess.stats,
               decision=res["decision"])
    sess.close()
    return out


def roofline(stats):
    legs = {"hist_large": stats.hist_large, "hist_small": stats.hist_small}
    name, k = max(legs.items(), key=lambda kv: kv[1].ms)
    if k.launches == 0 or k.ms <= 0:
        return None, None
    avg_ms = k.ms / k.launches
    bytes_per_launch = k.alg_bytes / k.launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": name, "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_launch": round(bytes_per_launch, 1),
            "launches": int(k.launches)}, {
        f: {"launches": int(getattr(stats, f).launches), "ms": round(getattr(stats, f).ms, 3),
            "alg_GB": round(getattr(stats, f).alg_bytes / 1e9, 4)}
        for f in ("hist_large", "hist_small", "finalize", "permut")}


def cpu_baseline(c, pr, mode):
    """The CPU oracle, unchanged, on one whole iteration (iteration 1, every
    tree) of the same workload, on all host threads.  Binning happens once
    per job; it is timed separately and left out, as on the GPU side."""
    import numpy as np
    from oracle import oracle as O
    cores = os.cpu_count() or 1
    X, y = c["X"], c["y"]
    p = X.shape[1]
    st = np.zeros(p, np.int8)
    ht = np.zeros(p, np.int32)
    t0 = time.perf_counter()
    O.bin_matrix(X, pr["n_bins"])
    t_bin = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.boruta_step(X, y, c["n_classes"], pr["n_trees"], pr["max_depth"], 1, st, ht,
                  mtry=pr["mtry"], importance_mode=mode, alpha=pr["alpha"], seed=c["seed"],
                  n_bins=pr["n_bins"], n_perm=pr["n_perm"], n_threads=cores, trace=False)
    t_iter = time.perf_counter() - t0 - t_bin
    return {"value": round(1.0 / t_iter, 5), "unit": "iters/s", "cores": cores,
            "kind": "oracle",
            "sample": f"one whole iteration (t=1, all {pr['n_trees']} trees, shadows, "
                      f"importance, decision) on {cores} threads: {t_iter:.2f}s; the once-per-"
                      f"job binning ({t_bin:.2f}s) is left out"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "design is described in DESIGN.md and is not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_09950_amd import binding as B
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()
    if args.probe_copy:
        probe_copy(args.probe_copy)
        return
    c, pr, n, p, desc = workload(args.workload)
    mode = B.TREEIMP if args.mode == "treeimp" else B.PERMUT
    # timed region: iterations replayed from the captured HIP graph
    main_leg = run_gpu(c, pr, mode, args.steps, args.warmup, B.FORM_BATCHED, B.RANK_FP32,
                       stats=False, graph=True)
    value = main_leg["steps"] / main_leg["seconds"]
    # the same iterations launched eagerly with HIP events around every
    # forest kernel: per-kernel durations and algorithmic bytes
    ev_leg = run_gpu(c, pr, mode, args.steps, args.warmup, B.FORM_BATCHED, B.RANK_FP32,
                     stats=True, graph=False)
    assert ev_leg["steps"] == main_leg["steps"]
    assert (ev_leg["decision"] == main_leg["decision"]).all()
    roof, kernels = roofline(ev_leg["stats"])
    extra = {"kernels": kernels, "timed_iterations": f"{args.warmup + 1}.."
             f"{args.warmup + main_leg['steps']}",
             "device_iter_ms": round(ev_leg["stats"].iter_ms / max(1, ev_leg["steps"]), 3),
             "eager_iters_per_s": round(ev_leg["steps"] / ev_leg["seconds"], 3)}
    st = ev_leg["stats"]
    extra["nodes_per_iteration_by_depth"] = {
        "small": [round(st.level_small[d] / main_leg["steps"], 1)
                  for d in range(pr["max_depth"])],
        "large": [round(st.level_large[d] / main_leg["steps"], 1)
                  for d in range(pr["max_depth"])]}
    if not args.no_compare:
        k = max(1, min(5, args.steps))
        other = B.PERMUT if mode == B.TREEIMP else B.TREEIMP
        leg = run_gpu(c, pr, other, k, args.warmup, B.FORM_BATCHED, B.RANK_FP32, stats=False)
        extra["other_mode_iters_per_s"] = round(leg["steps"] / leg["seconds"], 3)
        leg = run_gpu(c, pr, mode, k, args.warmup, B.FORM_BATCHED, B.RANK_EXACT, stats=False)
        extra["exact_rank_iters_per_s"] = round(leg["steps"] / leg["seconds"], 3)
        leg = run_gpu(c, pr, mode, 1, 1, B.FORM_PLAIN, B.RANK_FP32, stats=False)
        extra["plain_form_iters_per_s"] = round(leg["steps"] / leg["seconds"], 4)
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": main_leg["steps"], "warmup": args.warmup,
        "ms_per_step": round(1e3 * main_leg["seconds"] / main_leg["steps"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc + (", TreeImp" if mode == B.TREEIMP else ", Permut R=1") +
                   ", batched form, FP32 ranking + exact recheck", "n": n, "p": p,
                   "n_trees": pr["n_trees"], "max_depth": pr["max_depth"],
                   "n_bins": pr["n_bins"], "seed": c["seed"]},
        "roofline": roof,
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c, pr, mode)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
