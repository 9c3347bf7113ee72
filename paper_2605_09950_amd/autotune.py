"""Device-timed search over the launch parameters of the batched form.

The tunable parameters (boruta_options.small_rows, grid_small, grid_hist,
grid_finalize, col_level, col_unit, grid_col, and the histogram shapes
hist_rb / hist_rb_deep / band_level -- rows per lane per batch of the
node-major histogram for the large nodes of the first tree levels and for the
smaller nodes of the deeper ones --, hist_fw -- drawn features per histogram
item -- and col_waves -- wavefronts per workgroup of the column-major
histogram) change only how the work of a tree level is spread over
workgroups and lanes, which of the two split-search paths a node takes and
which of the two histogram layouts a level uses; every choice gives identical
results.  The search is a coordinate descent: each parameter in turn is set
to each of its candidate values, a session over the workload is stepped a few
times (graph replays, inputs resident on the device), and the fastest value
is kept.  The outcome can be cached in a text file, one line per workload
signature, which the library itself also reads (boruta_options.tune_cache).

    tune = autotune(jobs, n_bins=256)             # dict for Session(tune=...)
"""
import os
import time

import numpy as np

from paper_2605_09950_amd import binding as B

# candidate values per parameter, in search order (0 = library default).
# small_rows moves nodes between the two split-search kernels; it is left at
# the library default (32) unless the caller asks for it, so that per-kernel
# measurements stay comparable between tuned runs.
CANDIDATES = (
    ("col_level", (64, 5, 3, 7)),
    ("col_unit", (512, 4096)),
    ("grid_col", (1024, 4096)),
    ("col_waves", (8, 12)),
    ("hist_fw", (1, 2, 4)),
    ("hist_rb", (4, 16)),
    ("hist_rb_deep", (4, 16)),
    ("band_level", (3, 9)),
    ("grid_hist", (0, 4096, 32768, 65536)),
    ("grid_small", (0, 1024, 2048, 8192, 16384)),
    ("grid_finalize", (0, 1024, 2048, 8192)),
)
# the library's default of each parameter (boruta_default_options)
DEFAULTS = {"small_rows": 32, "col_unit": 2048, "hist_rb": 8, "hist_rb_deep": 8,
            "band_level": 6}


def signature(jobs, n_bins=256, n_perm=1):
    """Shape signature of a workload: what the launch parameters depend on (the
    same string the library computes for boruta_options.tune_cache)."""
    parts = [f"B{n_bins}", f"R{n_perm}"]
    for jd in jobs:
        n, p = jd["X"].shape
        k = "reg" if "y_reg" in jd else jd.get("n_classes", 2)
        parts.append(f"{n}x{p}K{k}T{jd['n_trees']}D{jd['max_depth']}"
                     f"m{jd.get('mtry', 0)}i{jd.get('importance_mode', 0)}")
    return "|".join(parts)


def read_cache(path):
    """{signature: tuning dict} of a cache file (missing file: empty)."""
    out = {}
    if not path or not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#") or "\t" not in line:
                continue
            sig, kv = line.split("\t", 1)
            out[sig] = {k: int(v) for k, v in (t.split("=", 1) for t in kv.split() if "=" in t)}
    return out


def write_cache(path, entries):
    with open(path, "w") as f:
        f.write("# launch tuning cache: workload signature, tab, key=value pairs\n")
        for sig, tune in sorted(entries.items()):
            f.write(sig + "\t" + " ".join(f"{k}={v}" for k, v in sorted(tune.items())) + "\n")


def _time_session(dev_jobs, shapes, n_bins, n_perm, tune, steps, warmup):
    """ms per job-iteration of `steps` iterations enqueued back to back
    (graph replays, no host wait between them) after `warmup` iterations."""
    import torch
    ws_bytes = B.boruta_workspace_size(shapes, n_bins=n_bins, n_perm=n_perm, tune=tune)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    with B.Session(dev_jobs, n_bins=n_bins, n_perm=n_perm, inputs_on_device=True,
                   workspace=ws, stream=stream, graph=True, tune=tune) as s:
        live = len(dev_jobs)
        if warmup:
            live, _ = s.run(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        if live:
            _, done = s.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return el / max(1, done) * 1e3


# a candidate replaces the best only when it is faster by more than this
# fraction (timing noise of short sessions)
MIN_GAIN = 0.01
# each timed session covers at least about this many milliseconds
SESSION_MS = 60.0


SMALL_ROWS = ("small_rows", (32, 64, 48, 16))


def autotune(jobs, n_bins=256, n_perm=1, steps=3, warmup=2, cache=None, log=None, report=None,
             tune_small_rows=False):
    """Returns the fastest tuning dict for `jobs` (host arrays, as for
    boruta_fit_batch).  With `cache` (a tuning cache file, the format
    boruta_options.tune_cache reads) a stored result for
    the same signature is reused and a new one is stored.  `report` (a dict)
    receives the number of timed sessions and their times."""
    import torch
    sig = signature(jobs, n_bins, n_perm)
    stored = read_cache(cache)
    if sig in stored:
        return dict(stored[sig])
    dev, shapes = [], []
    for jd in jobs:
        d = dict(jd)
        d["X"] = torch.from_numpy(np.ascontiguousarray(jd["X"])).cuda()
        for key in ("y", "y_reg"):
            if key in jd:
                d[key] = torch.from_numpy(np.ascontiguousarray(jd[key])).cuda()
        d["max_iter"] = min(jd.get("max_iter", 20), warmup + steps)
        dev.append(d)
        shapes.append(dict(n=d["X"].shape[0], p=d["X"].shape[1], regression="y_reg" in jd,
                           **{k: v for k, v in d.items() if k not in ("X", "y", "y_reg")}))
    best = {}
    best_ms = _time_session(dev, shapes, n_bins, n_perm, best, steps, warmup)
    # fast workloads: more iterations per session, so that each covers about
    # SESSION_MS of device time
    per_step = best_ms * len(dev)
    more = min(30, max(steps, int(np.ceil(SESSION_MS / max(per_step, 1e-3)))))
    if more > steps:
        steps = more
        for d, jd, sh in zip(dev, jobs, shapes):
            d["max_iter"] = sh["max_iter"] = min(jd.get("max_iter", 20), warmup + steps)
        best_ms = _time_session(dev, shapes, n_bins, n_perm, best, steps, warmup)
    trials = [({}, best_ms)]
    for key, values in ((SMALL_ROWS,) if tune_small_rows else ()) + CANDIDATES:
        for v in values:
            if best.get(key, DEFAULTS.get(key, 0)) == v:
                continue
            cand = dict(best, **{key: v})
            ms = _time_session(dev, shapes, n_bins, n_perm, cand, steps, warmup)
            trials.append((cand, ms))
            if log:
                log(f"autotune {cand}: {ms:.3f} ms/step")
            if ms < best_ms * (1.0 - MIN_GAIN):
                best, best_ms = cand, ms
    if best:
        # the choice against the defaults once more, back to back
        base_ms = _time_session(dev, shapes, n_bins, n_perm, {}, steps, warmup)
        again_ms = _time_session(dev, shapes, n_bins, n_perm, best, steps, warmup)
        trials += [({}, base_ms), (dict(best), again_ms)]
        if again_ms >= base_ms * (1.0 - MIN_GAIN):
            best = {}
    if report is not None:
        report["sessions"] = len(trials)
        report["steps"] = steps
        report["trials"] = [{"tune": t, "ms_per_step": round(m, 4)} for t, m in trials]
    if cache:
        stored = read_cache(cache)
        stored[sig] = best
        write_cache(cache, stored)
    return best
