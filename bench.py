"""Benchmark: Boruta iterations/s on one MI355X, with the histogram kernel's
algorithmic bandwidth against the HBM roofline and the CPU oracle beside it.

A step is one Boruta iteration (shadow widening, bootstrap, random forest,
importance, hits, decision) of every live job of the workload.  The default
workload is the MADELON-like one: n=10,000 rows, p=500 float32 features (20
informative, 80 noisy mixes, 400 noise), 3 classes, 256 quantile bins, 200
trees of depth 12, mtry = floor(sqrt(p_w)).  Inputs are resident in device
memory (torch tensors) before the timed region; binning happens once per
job, at session creation, outside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload madelon|planted|omics|manyjob|scale|regression]
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
    ap.add_argument("--mode", choices=["treeimp", "permut", "kl", "workload"], default="workload",
                    help="importance mode (default: the workload's own); kl = Algorithm 3's "
                         "prediction divergence")
    ap.add_argument("--workload", choices=["madelon", "planted", "omics", "manyjob", "scale",
                                           "regression"],
                    default="madelon")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other-mode / exact / plain comparison legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--set", default="", metavar="KEY=V,...",
                    help="launch tuning values (boruta_options fields), instead of the autotuner")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the device-timed autotuner (library default launch parameters)")
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
    """(jobs, run parameters, description, config keys) of a named workload."""
    from paper_2605_09950_amd import synth
    if name == "manyjob":
        cs = synth.many_jobs()
        pr = cs[0]["params"]
        desc = ("64 independent jobs, n in [200, 5000], p in [50, 2000], 2-5 classes, 256 "
                "bins, 100 trees depth 10 each, Permut R=1, each job's own seed")
        keys = {"jobs": 64, "n_trees": 100, "max_depth": 10, "n_bins": 256,
                "seeds": "8000+j"}
    else:
        idx = {"planted": 0, "madelon": 1, "omics": 2, "scale": 4, "regression": 5}[name]
        cs = [synth.config(idx)]
        pr = cs[0]["params"]
        n, p = cs[0]["X"].shape
        desc = {
            "planted": "planted n=500 p=20 K=2, 64 bins, 50 trees depth 8",
            "madelon": "MADELON-like n=10000 p=500 K=3 (20 informative, 80 mixes), 256 bins, "
                       "200 trees depth 12",
            "omics": "omics-shaped n=2000 p=20000 K=2 log-normal, 256 bins, 500 trees depth 12",
            "scale": "mixed-type n=100000 p=2000 K=4, 256 bins, 300 trees depth 16",
            "regression": "regression n=10000 p=50 U(0,1) (10 informative), float target, "
                          "256 bins, 200 trees depth 12",
        }[name]
        keys = {"n": n, "p": p, "n_trees": pr["n_trees"], "max_depth": pr["max_depth"],
                "n_bins": pr["n_bins"], "seed": cs[0]["seed"]}
    jobs = [dict({"y_reg": c["y_reg"]} if "y_reg" in c else
                 {"y": c["y"], "n_classes": c["n_classes"]},
                 X=c["X"], n_trees=c["params"]["n_trees"], max_depth=c["params"]["max_depth"],
                 mtry=c["params"]["mtry"], importance_mode=c["params"]["importance_mode"],
                 max_iter=c["params"]["max_iter"], alpha=c["params"]["alpha"], seed=c["seed"])
            for c in cs]
    return jobs, pr, desc, keys


def run_gpu(jobs, pr, steps, warmup, form, rank, stats, graph=True, tune=None):
    """A session over device-resident inputs and a torch workspace: `warmup`
    untimed steps, then up to `steps` timed ones.  Returns the timed
    job-iterations, seconds, stats and the final decisions."""
    import torch
    from paper_2605_09950_amd import binding as B
    dev, shapes = [], []
    torch.cuda.synchronize()
    t_up = time.perf_counter()  # host-to-device upload of the inputs (PCIe)
    for jd in jobs:
        d = dict(jd)
        d["X"] = torch.from_numpy(jd["X"]).cuda()
        for key in ("y", "y_reg"):
            if key in jd:
                d[key] = torch.from_numpy(jd[key]).cuda()
        d["max_iter"] = min(jd["max_iter"], 1000, warmup + steps)
        dev.append(d)
        shapes.append(dict(n=d["X"].shape[0], p=d["X"].shape[1], regression="y_reg" in jd,
                           **{k: v for k, v in d.items() if k not in ("X", "y", "y_reg")}))
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t_up
    ws_bytes = B.boruta_workspace_size(shapes, n_bins=pr["n_bins"], n_perm=pr["n_perm"],
                                       tune=tune)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    # session set-up: validation, labels, binning and the decision thresholds
    # of every job (inputs already on the device), outside the timed region
    sess = B.Session(dev, n_bins=pr["n_bins"], n_perm=pr["n_perm"], split_rank=rank,
                     form=form, stats=stats, inputs_on_device=True, workspace=ws,
                     stream=stream, graph=graph, tune=tune)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    live = len(jobs)
    for _ in range(warmup):
        if live:
            live = sess.step()
    torch.cuda.synchronize()
    if sess.stats is not None:  # count only the timed iterations
        for f in KERNELS:
            k = getattr(sess.stats, f)
            k.launches, k.ms, k.alg_bytes = 0, 0.0, 0.0
        sess.stats.iter_ms, sess.stats.iterations, sess.stats.nodes = 0.0, 0, 0
        sess.stats.permut_visits = 0.0
        for d in range(32):
            sess.stats.level_small[d] = sess.stats.level_large[d] = 0
    done, job_iters = 0, 0
    if graph and not stats:
        # the timed iterations enqueued back to back (graph replays, no host
        # wait between them); the steps run are read from the jobs afterwards
        before = [sess.result(j)["n_iter"] for j in range(len(jobs))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if live:
            live, job_iters = sess.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        done = max(sess.result(j)["n_iter"] - before[j] for j in range(len(jobs)))
    else:
        t0 = time.perf_counter()
        for _ in range(steps):
            if live == 0:
                break
            job_iters += live
            live = sess.step()
            done += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    decisions = [sess.result(j)["decision"] for j in range(len(jobs))]
    out = dict(steps=done, job_iters=job_iters, seconds=el, stats=sess.stats,
               decisions=decisions, setup_s=t_setup, upload_s=t_up)
    sess.close()
    return out


# kernel statistics of the library: node-major histogram (large nodes),
# wave path (small nodes), split/partition, OOB traversal, column-major histogram
KERNELS = ("hist_large", "hist_small", "finalize", "permut", "hist_col")
# the kernel behind each histogram statistic (for the counter summaries)
KERNEL_NAMES = {"hist_large": "k_hist_tile", "hist_small": "k_split_small",
                "hist_col": "k_hist_col"}


def roofline(stats):
    legs = {f: getattr(stats, f) for f in ("hist_large", "hist_small", "hist_col")}
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
        for f in KERNELS}


def measured_traffic(workload_name, kernel):
    """HBM-side traffic per launch of the histogram kernel (bytes), from the
    calibrated FETCH_SIZE + WRITE_SIZE counter summary committed under
    profiles/, or None when there is none for this workload or the kernel
    source has changed since the counters were taken."""
    if kernel not in KERNEL_NAMES:
        return None
    path = os.path.join(ROOT, "profiles", f"{KERNEL_NAMES[kernel]}_{workload_name}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith(("traffic_bytes_per_launch",
                                                        "kernel_code_sha256")):
                k, v = line.strip().split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_code_sha256") != kernel_code_digest() or \
            "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def kernel_code_digest():
    """SHA-256 of the code lines (line comments and blank lines dropped) of
    the forest kernels and their headers: the key under which a counter
    summary in profiles/ stays valid."""
    import hashlib
    lines = []
    for name in ("k_forest.hip", "forest_dev.hpp", "dev_common.hpp"):
        with open(os.path.join(ROOT, "paper_2605_09950_amd", "csrc", name)) as f:
            for line in f:
                code = line.split("//", 1)[0].rstrip()
                if code.strip():
                    lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def cpu_baseline(name, jobs, pr):
    """The CPU oracle, unchanged, on a bounded sample of the same workload on
    all host threads: whole iterations in sequence (MADELON-like, planted)
    until about 10 s have passed, a subset of the trees of iteration 1 scaled
    to the whole forest (omics-shaped, mixed-type), or whole first iterations
    of a subset of the jobs (many-job).  Binning happens once per job; it is
    timed separately and left out, as on the GPU side."""
    import numpy as np
    from oracle import oracle as O
    cores = os.cpu_count() or 1

    def step(jd, t, st, ht, trees=None, threads=cores):
        return O.boruta_step(jd["X"], jd["y"], jd["n_classes"], jd["n_trees"],
                             jd["max_depth"], t, st, ht, mtry=jd["mtry"],
                             importance_mode=jd["importance_mode"], alpha=jd["alpha"],
                             seed=jd["seed"], n_bins=pr["n_bins"], n_perm=pr["n_perm"],
                             tree_subset=trees, n_threads=threads, trace=False)

    def bin_time(jd):
        t0 = time.perf_counter()
        O.bin_matrix(jd["X"], pr["n_bins"])
        return time.perf_counter() - t0

    if name in ("madelon", "planted"):
        jd = jobs[0]
        p = jd["X"].shape[1]
        st, ht = np.zeros(p, np.int8), np.zeros(p, np.int32)
        t_bin, spent, it = bin_time(jd), 0.0, 0
        while spent < 10.0 and it < jd["max_iter"]:
            t0 = time.perf_counter()
            r = step(jd, it + 1, st, ht)
            spent += time.perf_counter() - t0 - t_bin
            st, ht, it = r["state"], r["hits"], it + 1
        # one core: the first trees of iteration 1 on one thread, scaled to the forest
        k = min(jd["n_trees"], 8)
        t0 = time.perf_counter()
        step(jd, 1, np.zeros(p, np.int8), np.zeros(p, np.int32), list(range(k)), threads=1)
        one = time.perf_counter() - t0 - t_bin
        return {"value": round(it / spent, 5), "unit": "iters/s", "cores": cores,
                "kind": "oracle",
                "sample": f"iterations 1..{it} in sequence (all {jd['n_trees']} trees each) on "
                          f"{cores} threads: {spent:.2f}s; the once-per-job binning "
                          f"({t_bin:.2f}s per call) is left out",
                "one_core": {"value": round(k / (one * jd["n_trees"]), 5), "unit": "iters/s",
                             "sample": f"trees 0..{k - 1} of iteration 1 on one thread in "
                                       f"{one:.2f}s, scaled by {jd['n_trees']}/{k}"}}
    if name == "regression":
        jd = jobs[0]
        t_bin = bin_time(jd)
        t0 = time.perf_counter()
        O.boruta_fit_reg(jd["X"], jd["y_reg"], jd["n_trees"], jd["max_depth"], max_iter=1,
                         seed=jd["seed"], n_bins=pr["n_bins"], n_threads=cores)
        one_it = max(1e-3, time.perf_counter() - t0 - t_bin)
        it = int(max(1, min(jd["max_iter"], 10.0 // one_it)))
        t0 = time.perf_counter()
        r = O.boruta_fit_reg(jd["X"], jd["y_reg"], jd["n_trees"], jd["max_depth"], max_iter=it,
                             seed=jd["seed"], n_bins=pr["n_bins"], n_threads=cores)
        spent = time.perf_counter() - t0 - t_bin
        # one core: iteration 1 on one thread
        t0 = time.perf_counter()
        O.boruta_fit_reg(jd["X"], jd["y_reg"], jd["n_trees"], jd["max_depth"], max_iter=1,
                         seed=jd["seed"], n_bins=pr["n_bins"], n_threads=1)
        one = max(1e-3, time.perf_counter() - t0 - t_bin)
        return {"value": round(r["n_iter"] / spent, 5), "unit": "iters/s", "cores": cores,
                "kind": "oracle",
                "sample": f"iterations 1..{r['n_iter']} in sequence (all {jd['n_trees']} "
                          f"trees each) on {cores} threads: {spent:.2f}s; the binning "
                          f"({t_bin:.2f}s) is left out",
                "one_core": {"value": round(1.0 / one, 5), "unit": "iters/s",
                             "sample": f"iteration 1 (all {jd['n_trees']} trees) on one "
                                       f"thread in {one:.2f}s"}}
    if name in ("omics", "scale"):
        jd = jobs[0]
        p = jd["X"].shape[1]
        k = min(jd["n_trees"], cores)
        trees = list(range(k))
        t_bin = bin_time(jd)
        t0 = time.perf_counter()
        step(jd, 1, np.zeros(p, np.int8), np.zeros(p, np.int32), trees)
        spent = time.perf_counter() - t0 - t_bin
        it_time = spent * jd["n_trees"] / k
        return {"value": round(1.0 / it_time, 6), "unit": "iters/s", "cores": cores,
                "kind": "oracle",
                "sample": f"trees 0..{k - 1} of iteration 1 (one per thread, {cores} threads) "
                          f"in {spent:.2f}s, scaled by {jd['n_trees']}/{k} to the whole forest; "
                          f"binning ({t_bin:.2f}s) left out"}
    # many-job: first iterations of the first jobs until about 10 s have passed
    spent, done = 0.0, 0
    for jd in jobs:
        if spent >= 10.0:
            break
        p = jd["X"].shape[1]
        t_bin = bin_time(jd)
        t0 = time.perf_counter()
        step(jd, 1, np.zeros(p, np.int8), np.zeros(p, np.int32))
        spent += time.perf_counter() - t0 - t_bin
        done += 1
    return {"value": round(done / spent, 5), "unit": "job-iters/s", "cores": cores,
            "kind": "oracle",
            "sample": f"iteration 1 of jobs 0..{done - 1} (all 100 trees each, {cores} threads "
                      f"per job) in {spent:.2f}s; binning left out"}


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
    jobs, pr, desc, keys = workload(args.workload)
    if args.mode != "workload":
        for jd in jobs:
            jd["importance_mode"] = {"treeimp": B.TREEIMP, "permut": B.PERMUT,
                                     "kl": B.PERMUT_KL}[args.mode]
    mode = jobs[0]["importance_mode"]
    unit = "job-iters/s" if len(jobs) > 1 else "iters/s"
    tune, tune_s, tune_report = None, 0.0, {}
    if args.set:
        tune = {k: int(v) for k, v in (kv.split("=") for kv in args.set.split(","))}
    elif not args.no_tune:  # results are identical for every choice; timed outside the region
        from paper_2605_09950_amd.autotune import autotune
        t0 = time.perf_counter()
        tune = autotune(jobs, n_bins=pr["n_bins"], n_perm=pr["n_perm"], report=tune_report)
        tune_s = time.perf_counter() - t0
    # timed region: iterations replayed from the captured HIP graph
    main_leg = run_gpu(jobs, pr, args.steps, args.warmup, B.FORM_BATCHED, B.RANK_FP32,
                       stats=False, graph=True, tune=tune)
    value = main_leg["job_iters"] / main_leg["seconds"]
    # the same iterations launched eagerly with HIP events around every
    # forest kernel: per-kernel durations and algorithmic bytes
    ev_leg = run_gpu(jobs, pr, args.steps, args.warmup, B.FORM_BATCHED, B.RANK_FP32,
                     stats=True, graph=False, tune=tune)
    assert ev_leg["job_iters"] == main_leg["job_iters"]
    assert all((a == b).all() for a, b in zip(ev_leg["decisions"], main_leg["decisions"]))
    roof, kernels = roofline(ev_leg["stats"])
    if roof is not None:
        roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    st = ev_leg["stats"]
    n_steps = max(1, ev_leg["steps"])
    extra = {"kernels": kernels, "timed_iterations": f"{args.warmup + 1}.."
             f"{args.warmup + main_leg['steps']}", "job_iterations": main_leg["job_iters"],
             "device_iter_ms": round(st.iter_ms / n_steps, 3),
             # per run, before the iterations: validation, labels, binning
             "setup_ms_binning": round(main_leg["setup_s"] * 1e3, 2),
             "upload_ms_pcie": round(main_leg["upload_s"] * 1e3, 2),
             "tune": dict(tune or {}, **({"search_s": round(tune_s, 2),
                                          "sessions": tune_report.get("sessions", 0)}
                                         if tune is not None else {})),
             "eager_" + unit.replace("/", "_per_"): round(ev_leg["job_iters"] /
                                                         ev_leg["seconds"], 3),
             # Permut's out-of-bag walks: tree nodes visited per second of its kernel
             "permut_node_visits_per_s": (round(st.permut_visits / (st.permut.ms * 1e-3), 1)
                                          if st.permut.ms > 0 else None),
             "nodes_per_step_by_depth": {
                 "small": [round(st.level_small[d] / n_steps, 1)
                           for d in range(max(j["max_depth"] for j in jobs))],
                 "large": [round(st.level_large[d] / n_steps, 1)
                           for d in range(max(j["max_depth"] for j in jobs))]}}
    regression = any("y_reg" in jd for jd in jobs)
    if not args.no_compare:
        k = max(1, min(5, args.steps))
        if not regression:  # the regression forest has TreeImp only
            other = [dict(jd, importance_mode=B.PERMUT if jd["importance_mode"] == B.TREEIMP
                          else B.TREEIMP) for jd in jobs]
            leg = run_gpu(other, pr, k, args.warmup, B.FORM_BATCHED, B.RANK_FP32,
                          stats=False, tune=tune)
            extra["other_mode_" + unit.replace("/", "_per_")] = round(
                leg["job_iters"] / leg["seconds"], 3)
        if mode != B.PERMUT_KL and not regression:
            kl = [dict(jd, importance_mode=B.PERMUT_KL) for jd in jobs]
            leg = run_gpu(kl, pr, k, args.warmup, B.FORM_BATCHED, B.RANK_FP32, stats=False,
                          tune=tune)
            extra["permut_kl_" + unit.replace("/", "_per_")] = round(
                leg["job_iters"] / leg["seconds"], 3)
        leg = run_gpu(jobs, pr, k, args.warmup, B.FORM_BATCHED, B.RANK_EXACT, stats=False,
                      tune=tune)
        extra["exact_rank_" + unit.replace("/", "_per_")] = round(
            leg["job_iters"] / leg["seconds"], 3)
        if args.workload == "scale":
            # one launch per node: about a million launches per iteration here
            extra["plain_form_note"] = "not run on this workload (one launch per tree node)"
        else:
            leg = run_gpu(jobs, pr, 1, 1, B.FORM_PLAIN, B.RANK_FP32, stats=False)
            extra["plain_form_" + unit.replace("/", "_per_")] = round(
                leg["job_iters"] / leg["seconds"], 4)
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": unit, "n_gpus": 1,
        "steps": main_leg["steps"], "warmup": args.warmup,
        "ms_per_step": round(1e3 * main_leg["seconds"] / max(1, main_leg["steps"]), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": dict({"workload": desc + {B.TREEIMP: ", TreeImp",
                                            B.PERMUT: f", Permut R={pr['n_perm']}",
                                            B.PERMUT_KL: ", Permut-KL (Algorithm 3)"}[mode] +
                        ", batched form, FP32 ranking + exact recheck"}, **keys),
        "roofline": roof,
        "extra": extra,
    }
    if mode == B.PERMUT_KL:
        # the oracle's divergence step re-routes every (column, row, tree): no
        # sample of it stays within the CPU leg's time budget
        extra["cpu_baseline_note"] = "not run for the divergence mode"
    elif not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, jobs, pr)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
