"""Benchmark: Boruta iterations/s on one MI355X, with the histogram kernel's
algorithmic bandwidth against the HBM roofline and the CPU oracle beside it.

A step is one Boruta iteration (shadow widening, bootstrap, random forest,
importance, hits, decision) of every live job of the workload.  The default
workload is the mixed-type one, the largest that one GPU holds: n=100,000
rows, p=2,000 float32 features (45% N(0,1), 45% U(0,1), 10% categorical
codes; 40 informative), 4 classes from a random depth-6 tree, 256 quantile
bins, 300 trees of depth 16, mtry = floor(sqrt(p_w)), TreeImp; its widened
bin matrix (400 MB) exceeds the 256 MB last-level cache.  Inputs are resident
in device memory (torch tensors) before the timed region; binning happens
once per job, at session creation, outside it.

Besides the timed batched/FP32-ranked leg the line carries: an event-timed
eager leg (per-kernel durations, algorithmic bytes: the roofline), the
library's streaming-copy bandwidth (the attainable figure), the exact-only
ranking and the plain per-node form (both checked equal to the FP32 leg), the
other importance mode, Algorithm 3's divergence mode, the MADELON-like
workload's rate, roofline and whole-run time, and the CPU oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload scale|madelon|planted|omics|manyjob|regression]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

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
                    default="scale")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other-mode / exact / plain comparison legs")
    ap.add_argument("--no-madelon", action="store_true",
                    help="skip the MADELON-like legs reported beside another workload")
    ap.add_argument("--profile-leg", action="store_true",
                    help="run only the event-timed leg (no warmup) and print its per-kernel "
                         "launches and algorithmic bytes: the command that hardware counters "
                         "are collected over")
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
        d["X"] = torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda()
        for key in ("y", "y_reg"):
            if key in jd:
                d[key] = torch.from_numpy(np.ascontiguousarray(jd[key])).cuda()
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
    results = [sess.result(j) for j in range(len(jobs))]
    out = dict(steps=done, job_iters=job_iters, seconds=el, stats=sess.stats,
               decisions=[r["decision"] for r in results], results=results, setup_s=t_setup,
               upload_s=t_up)
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


def counter_summary(workload_name, kernel):
    """The machine-read fields of the calibrated FETCH_SIZE + WRITE_SIZE
    counter summary committed under profiles/ for this kernel and workload:
    traffic per launch (bytes) and the algorithmic bytes per launch of the
    same launches; None when there is none, or when the kernel source has
    changed since the counters were taken."""
    if kernel not in KERNEL_NAMES:
        return None
    path = os.path.join(ROOT, "profiles", f"{KERNEL_NAMES[kernel]}_{workload_name}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith(("traffic_bytes_per_launch",
                                                        "kernel_code_sha256",
                                                        "alg_bytes_per_launch")):
                k, v = line.strip().split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_code_sha256") != kernel_code_digest() or \
            "traffic_bytes_per_launch" not in fields:
        return None
    out = {"traffic": float(fields["traffic_bytes_per_launch"])}
    if "alg_bytes_per_launch" in fields:
        out["alg"] = float(fields["alg_bytes_per_launch"])
    return out


def measured_traffic(workload_name, kernel):
    """HBM-side traffic per launch of the histogram kernel (bytes), or None
    (see counter_summary)."""
    c = counter_summary(workload_name, kernel)
    return None if c is None else c["traffic"]


def copy_bandwidth(nbytes=1 << 30, launches=10):
    """Attainable HBM bandwidth: the library's streaming copy kernel over
    nbytes (read once, written once) timed with HIP events on the launching
    stream; GB/s of read + write bytes."""
    import torch
    from paper_2605_09950_amd import binding as B
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    B.boruta_probe_copy(dst, src, nbytes, stream=st)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(launches):
        B.boruta_probe_copy(dst, src, nbytes, stream=st)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    del src, dst
    return {"GB_per_s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "bytes": nbytes,
            "launches": launches, "avg_launch_ms": round(ms, 4)}


def kernel_code_digest():
    """SHA-256 of the code lines (line comments and blank lines dropped) of
    the forest kernels and their headers: the key under which a counter
    summary in profiles/ stays valid."""
    import hashlib
    lines = []
    for name in ("k_forest.hip", "forest_dev.hpp", "dev_common.hpp", "reg_dev.hpp"):
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


def same_results(a, b, iters):
    """Equal decisions, hits, and history and shadow maxima of the first
    `iters` iterations, job by job (the history holds the exact integer
    importances divided once in IEEE double, so equal rows mean equal
    integers)."""
    for ra, rb in zip(a["results"], b["results"]):
        k = min(iters, ra["n_iter"], rb["n_iter"])
        ha, hb = ra["imp_history"][:k], rb["imp_history"][:k]
        if not (np.array_equal(np.isnan(ha), np.isnan(hb)) and
                np.array_equal(ha[~np.isnan(ha)], hb[~np.isnan(hb)]) and
                np.array_equal(ra["shadow_max"][:k], rb["shadow_max"][:k])):
            return False
        if ra["n_iter"] == rb["n_iter"] and not (
                np.array_equal(ra["decision"], rb["decision"]) and
                np.array_equal(ra["hits"], rb["hits"])):
            return False
    return True


def rate(leg):
    return round(leg["job_iters"] / leg["seconds"], 4) if leg["seconds"] > 0 else None


def roofline_legs(jobs, pr, steps, warmup, tune, workload_name):
    """The timed graph leg and the event-timed eager leg of one workload;
    returns (main leg, event leg, roofline dict, per-kernel figures)."""
    from paper_2605_09950_amd import binding as B
    main_leg = run_gpu(jobs, pr, steps, warmup, B.FORM_BATCHED, B.RANK_FP32, stats=False,
                       graph=True, tune=tune)
    ev_leg = run_gpu(jobs, pr, steps, warmup, B.FORM_BATCHED, B.RANK_FP32, stats=True,
                     graph=False, tune=tune)
    assert ev_leg["job_iters"] == main_leg["job_iters"]
    assert same_results(ev_leg, main_leg, warmup + steps), "event leg differs from graph leg"
    roof, kernels = roofline(ev_leg["stats"])
    if roof is not None:
        c = counter_summary(workload_name, roof["kernel"])
        roof["traffic"] = None if c is None else c["traffic"]
        if c is not None and c.get("alg"):
            # waste ratio of the profiled launches (traffic and algorithmic
            # bytes of the same iterations)
            roof["traffic_over_alg"] = round(c["traffic"] / c["alg"], 3)
    return main_leg, ev_leg, roof, kernels


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); a run over "
              "several GPUs (trees split across them, one all-reduce of the integer "
              "importances per iteration) is not built.", file=sys.stderr)
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
    ukey = unit.replace("/", "_per_")
    tune, tune_s, tune_report = None, 0.0, {}
    if args.set:
        tune = {k: int(v) for k, v in (kv.split("=") for kv in args.set.split(","))}
    elif not args.no_tune:  # results are identical for every choice; timed outside the region
        from paper_2605_09950_amd.autotune import autotune
        t0 = time.perf_counter()
        tune = autotune(jobs, n_bins=pr["n_bins"], n_perm=pr["n_perm"], report=tune_report)
        tune_s = time.perf_counter() - t0
    if args.profile_leg:
        # the counters' command: exactly the event leg's launches, no warmup
        leg = run_gpu(jobs, pr, args.steps, 0, B.FORM_BATCHED, B.RANK_FP32, stats=True,
                      graph=False, tune=tune)
        st = leg["stats"]
        print(json.dumps({"profile_leg": args.workload, "steps": leg["steps"], "tune": tune,
                          "device_iter_ms": round(st.iter_ms / max(1, leg["steps"]), 3),
                          "kernels": {f: {"launches": int(getattr(st, f).launches),
                                          "ms": round(getattr(st, f).ms, 3),
                                          "alg_bytes_per_launch":
                                              getattr(st, f).alg_bytes /
                                              max(1, getattr(st, f).launches)}
                                      for f in KERNELS}}), flush=True)
        return
    # timed region: iterations replayed from the captured HIP graph; then the
    # same iterations launched eagerly with HIP events around every forest
    # kernel (per-kernel durations and algorithmic bytes)
    main_leg, ev_leg, roof, kernels = roofline_legs(jobs, pr, args.steps, args.warmup, tune,
                                                    args.workload)
    value = main_leg["job_iters"] / main_leg["seconds"]
    copy = copy_bandwidth()
    if roof is not None:
        roof["attainable_GBs"] = copy["GB_per_s"]
        roof["frac_of_attainable"] = round(roof["achieved"] / copy["GB_per_s"], 4)
    st = ev_leg["stats"]
    n_steps = max(1, ev_leg["steps"])
    extra = {"kernels": kernels, "timed_iterations": f"{args.warmup + 1}.."
             f"{args.warmup + main_leg['steps']}", "job_iterations": main_leg["job_iters"],
             "device_iter_ms": round(st.iter_ms / n_steps, 3),
             # per run, before the iterations: validation, labels, binning
             "setup_ms_binning": round(main_leg["setup_s"] * 1e3, 2),
             "upload_ms_pcie": round(main_leg["upload_s"] * 1e3, 2),
             "copy_probe": copy,
             "tune": dict(tune or {}, **({"search_s": round(tune_s, 2),
                                          "sessions": tune_report.get("sessions", 0)}
                                         if tune is not None else {})),
             "eager_" + ukey: round(ev_leg["job_iters"] / ev_leg["seconds"], 3),
             # Permut's out-of-bag walks: tree nodes visited per second of its kernel
             "permut_node_visits_per_s": (round(st.permut_visits / (st.permut.ms * 1e-3), 1)
                                          if st.permut.ms > 0 else None),
             "nodes_per_step_by_depth": {
                 "small": [round(st.level_small[d] / n_steps, 1)
                           for d in range(max(j["max_depth"] for j in jobs))],
                 "large": [round(st.level_large[d] / n_steps, 1)
                           for d in range(max(j["max_depth"] for j in jobs))]}}
    if not args.no_compare:
        k, w = max(1, min(3, args.steps)), args.warmup
        # the reference for the equality checks: the same iterations, FP32 ranking
        ref = run_gpu(jobs, pr, k, w, B.FORM_BATCHED, B.RANK_FP32, stats=False, tune=tune)
        leg = run_gpu(jobs, pr, k, w, B.FORM_BATCHED, B.RANK_EXACT, stats=False, tune=tune)
        assert same_results(leg, ref, w + k), "exact-only ranking differs from FP32 ranking"
        extra["exact_rank_" + ukey] = rate(leg)
        extra["exact_rank_equal_to_fp32"] = f"iterations 1..{w + k}: identical"
        # the plain per-node form: one launch per tree node, iteration 1
        leg = run_gpu(jobs, pr, 1, 0, B.FORM_PLAIN, B.RANK_FP32, stats=False)
        assert same_results(leg, ref, 1), "plain per-node form differs from the batched form"
        extra["plain_form_" + ukey] = rate(leg)
        extra["plain_form_note"] = ("iteration 1, one launch per tree node (histogram and "
                                    "split/partition launches per large node), identical "
                                    "to the batched form")
        other = [dict(jd, importance_mode=B.PERMUT if jd["importance_mode"] == B.TREEIMP
                      else B.TREEIMP) for jd in jobs]
        leg = run_gpu(other, pr, k, w, B.FORM_BATCHED, B.RANK_FP32, stats=False, tune=tune)
        extra["other_mode_" + ukey] = rate(leg)
        extra["other_mode"] = ("Permut" if other[0]["importance_mode"] == B.PERMUT
                               else "TreeImp") + f", R={pr['n_perm']}"
        if mode != B.PERMUT_KL:
            kl = [dict(jd, importance_mode=B.PERMUT_KL) for jd in jobs]
            leg = run_gpu(kl, pr, k, w, B.FORM_BATCHED, B.RANK_FP32, stats=False, tune=tune)
            extra["permut_kl_" + ukey] = rate(leg)
    if args.workload != "madelon" and not args.no_madelon:
        extra["madelon"] = madelon_legs()
    if len(jobs) == 1 and not args.no_compare:
        # the whole run of this workload, as the paper reports per run
        extra["whole_run"] = whole_run(jobs[0], pr, tune)
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


def madelon_legs():
    """The MADELON-like workload beside the headline: its iteration rate and
    roofline over iterations 3..22 (library defaults, no tuning), and one
    whole run (iterations until every feature is decided or 100) timed on the
    host clock, the quantity the paper's tables report per run."""
    import torch
    from paper_2605_09950_amd import binding as B
    jobs, pr, desc, _ = workload("madelon")
    main_leg, _, roof, _ = roofline_legs(jobs, pr, 20, 2, None, "madelon")
    return {"workload": desc + ", TreeImp", "iters_per_s": round(rate(main_leg), 3),
            "roofline": roof, "whole_run": whole_run(jobs[0], pr, None)}


def whole_run(jd, pr, tune):
    """One job's whole run (iterations until every feature is decided or
    max_iter) on device-resident inputs, timed on the host clock from the
    session's set-up: the quantity the paper's tables report per run."""
    import torch
    from paper_2605_09950_amd import binding as B
    d = dict(jd, X=torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda())
    for key in ("y", "y_reg"):  # classification labels or regression targets
        if key in jd:
            d[key] = torch.from_numpy(np.ascontiguousarray(jd[key])).cuda()
    dev = [d]
    shapes = [dict(n=d["X"].shape[0], p=d["X"].shape[1], regression="y_reg" in jd,
                   **{k: v for k, v in d.items() if k not in ("X", "y", "y_reg")})]
    ws = torch.empty(B.boruta_workspace_size(shapes, n_bins=pr["n_bins"], n_perm=pr["n_perm"],
                                             tune=tune),
                     dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with B.Session(dev, n_bins=pr["n_bins"], n_perm=pr["n_perm"], inputs_on_device=True,
                   workspace=ws, stream=torch.cuda.current_stream(), tune=tune) as s:
        t1 = time.perf_counter()
        _, its = s.run(jd["max_iter"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r = s.result(0)
    return {"iterations": int(its), "seconds": round(t2 - t0, 4),
            "set_up_seconds": round(t1 - t0, 4),
            "confirmed": int((r["decision"] == 1).sum()),
            "rejected": int((r["decision"] == -1).sum()),
            "tentative": int((r["decision"] == 0).sum())}


if __name__ == "__main__":
    main()
