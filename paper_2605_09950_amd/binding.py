"""ctypes binding of libboruta.so (include/boruta.h): same entry-point names,
argument marshalling only.  Every step of the method runs in the library's
HIP kernels; there is no Python or CPU fallback, and loading fails loudly
when the library has not been built."""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libboruta.so")

BORUTA_OK, BORUTA_E_INVALID_ARG, BORUTA_E_NONFINITE, BORUTA_E_OOM, BORUTA_E_DEVICE, \
    BORUTA_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
TREEIMP, PERMUT, PERMUT_KL = 0, 1, 2
FORM_PLAIN, FORM_BATCHED = 0, 1
RANK_EXACT, RANK_FP32 = 0, 1


class BorutaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libboruta error {code}: {msg}")
        self.code = code


class IterTrace(ctypes.Structure):
    _fields_ = [
        ("job", ctypes.c_int32), ("t", ctypes.c_int32), ("p_cur", ctypes.c_int32),
        ("n_sha", ctypes.c_int32), ("p_w", ctypes.c_int32), ("mtry", ctypes.c_int32),
        ("n_trees", ctypes.c_int32),
        ("col_src", ctypes.POINTER(ctypes.c_int32)),
        ("imp_int", ctypes.POINTER(ctypes.c_int64)),
        ("hits", ctypes.POINTER(ctypes.c_int32)),
        ("state", ctypes.POINTER(ctypes.c_int8)),
        ("tree_stats", ctypes.POINTER(ctypes.c_int64)),
        ("n_nodes", ctypes.c_int64),
        ("nodes", ctypes.POINTER(ctypes.c_int64)),
    ]


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(IterTrace))


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("hist_large", KernelStat), ("hist_small", KernelStat), ("finalize", KernelStat),
                ("permut", KernelStat),
                ("iter_ms", ctypes.c_double), ("iterations", ctypes.c_int64),
                ("nodes", ctypes.c_int64), ("level_small", ctypes.c_int64 * 32),
                ("level_large", ctypes.c_int64 * 32), ("hist_col", KernelStat),
                ("permut_visits", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("n_perm", ctypes.c_int32),
                ("split_rank", ctypes.c_int32), ("form", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("small_rows", ctypes.c_int32),
                ("grid_small", ctypes.c_int32), ("grid_hist", ctypes.c_int32),
                ("grid_finalize", ctypes.c_int32),
                ("col_level", ctypes.c_int32),
                ("col_unit", ctypes.c_int32),
                ("grid_col", ctypes.c_int32),
                ("kl_rows", ctypes.c_int32),
                ("perc", ctypes.c_int32), ("rough_fix", ctypes.c_int32),
                ("trace", TRACE_FN), ("trace_user", ctypes.c_void_p),
                ("stats", ctypes.POINTER(Stats)),
                ("hist_rb", ctypes.c_int32), ("hist_rb_deep", ctypes.c_int32),
                ("band_level", ctypes.c_int32), ("hist_fw", ctypes.c_int32),
                ("col_waves", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


class Job(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("p", ctypes.c_int64), ("n_classes", ctypes.c_int32),
                ("n_trees", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("mtry", ctypes.c_int32), ("importance_mode", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("y_reg", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("decision", ctypes.c_void_p), ("imp_history", ctypes.c_void_p),
                ("hits", ctypes.c_void_p), ("shadow_max", ctypes.c_void_p),
                ("rank", ctypes.c_void_p),
                ("n_iter", ctypes.c_int32), ("status", ctypes.c_int32)]


EXPORTS = ["boruta_default_options", "boruta_fit", "boruta_fit_ex", "boruta_fit_batch",
           "boruta_fit_seeds", "boruta_fit_seeds_regression", "boruta_fit_regression",
           "boruta_workspace_size", "boruta_fit_device", "boruta_fit_device_noalloc",
           "boruta_session_create",
           "boruta_session_step", "boruta_session_run", "boruta_session_result",
           "boruta_session_resume", "boruta_bin",
           "boruta_session_destroy", "boruta_probe_copy", "boruta_last_error"]

_lib = None


def lib():
    """Load libboruta.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7,
        # and a second copy loaded next to it cannot initialise the device.
        # Importing torch first lets libboruta bind to torch's runtime (same
        # SONAME), so torch tensors/streams and the library share it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_09950_amd.csrc.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint64, ctypes.c_double)
        prob = [P, P, i64, i64, i32, i32, i32, i32, i32, i32, f64, u64]
        L.boruta_default_options.argtypes = [ctypes.POINTER(Options)]
        L.boruta_default_options.restype = None
        L.boruta_fit.argtypes = prob + [P, P, P, P, P]
        L.boruta_fit.restype = ctypes.c_int
        L.boruta_fit_ex.argtypes = prob + [ctypes.POINTER(Options), P, P, P, P, P]
        L.boruta_fit_ex.restype = ctypes.c_int
        L.boruta_fit_batch.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(Options),
                                       ctypes.POINTER(Result)]
        L.boruta_fit_batch.restype = ctypes.c_int
        L.boruta_fit_regression.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, f64, u64,
                                            ctypes.POINTER(Options), P, P, P, P, P]
        L.boruta_fit_regression.restype = ctypes.c_int
        L.boruta_fit_seeds.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, i32, f64, P,
                                       i32, ctypes.POINTER(Options), P, P,
                                       ctypes.POINTER(Result)]
        L.boruta_fit_seeds.restype = ctypes.c_int
        L.boruta_fit_seeds_regression.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, f64,
                                                  P, i32, ctypes.POINTER(Options), P, P,
                                                  ctypes.POINTER(Result)]
        L.boruta_fit_seeds_regression.restype = ctypes.c_int
        L.boruta_workspace_size.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(Options),
                                            ctypes.POINTER(ctypes.c_size_t)]
        L.boruta_workspace_size.restype = ctypes.c_int
        L.boruta_fit_device.argtypes = prob + [ctypes.POINTER(Options), P, ctypes.c_size_t, P,
                                               P, P, P, P, P]
        L.boruta_fit_device.restype = ctypes.c_int
        L.boruta_fit_device_noalloc.argtypes = prob + [ctypes.POINTER(Options), P, P, P, P, P,
                                                       P]
        L.boruta_fit_device_noalloc.restype = ctypes.c_int
        L.boruta_session_create.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(Options),
                                            i32, P, ctypes.c_size_t, P,
                                            ctypes.POINTER(ctypes.c_void_p)]
        L.boruta_session_create.restype = ctypes.c_int
        L.boruta_session_step.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.boruta_session_step.restype = ctypes.c_int
        L.boruta_session_run.argtypes = [P, i32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.boruta_session_run.restype = ctypes.c_int
        L.boruta_session_result.argtypes = [P, i32, ctypes.POINTER(Result)]
        L.boruta_session_result.restype = ctypes.c_int
        L.boruta_session_resume.argtypes = [P, i32, i32, P, P]
        L.boruta_session_resume.restype = ctypes.c_int
        L.boruta_session_destroy.argtypes = [P]
        L.boruta_session_destroy.restype = None
        L.boruta_bin.argtypes = [P, i64, i64, i32, P]
        L.boruta_bin.restype = ctypes.c_int
        L.boruta_probe_copy.argtypes = [P, P, ctypes.c_size_t, P]
        L.boruta_probe_copy.restype = ctypes.c_int
        L.boruta_last_error.argtypes = []
        L.boruta_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def boruta_last_error():
    return lib().boruta_last_error().decode()


def _check(rc):
    if rc != BORUTA_OK:
        raise BorutaError(rc, boruta_last_error())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def boruta_default_options():
    o = Options()
    lib().boruta_default_options(ctypes.byref(o))
    return o


def _trace_collector(store, p, keep_iters=None):
    """Copies each iteration record into store["iters"] (only iterations in
    keep_iters when given).  p: the feature count, or one per job."""
    ps = list(p) if isinstance(p, (list, tuple)) else None

    def cb(_user, trp):
        tr = trp.contents
        p = ps[tr.job] if ps is not None else p0
        p_w, nt, nn = tr.p_w, tr.n_trees, tr.n_nodes
        if keep_iters is not None and tr.t not in keep_iters:
            return
        sink = store["sink"] if "sink" in store else store["iters"].append
        sink({
            "hits": np.ctypeslib.as_array(tr.hits, (p,)).copy(),
            "state": np.ctypeslib.as_array(tr.state, (p,)).copy(),
            "job": tr.job, "t": tr.t, "p_cur": tr.p_cur, "n_sha": tr.n_sha, "p_w": p_w,
            "mtry": tr.mtry,
            "col_src": np.ctypeslib.as_array(tr.col_src, (p_w,)).copy(),
            "imp_int": np.ctypeslib.as_array(tr.imp_int, (p_w,)).copy(),
            "tree_stats": np.ctypeslib.as_array(tr.tree_stats, (nt, 5)).copy(),
            "nodes": np.ctypeslib.as_array(tr.nodes, (nn, 6)).copy() if nn else
            np.zeros((0, 6), np.int64),
        })
    p0 = p
    return TRACE_FN(cb)


TUNE_KEYS = ("small_rows", "grid_small", "grid_hist", "grid_finalize", "col_level", "col_unit",
             "grid_col", "kl_rows", "hist_rb", "hist_rb_deep", "band_level", "hist_fw",
             "col_waves")


def make_options(n_bins=256, n_perm=1, split_rank=RANK_FP32, form=FORM_BATCHED, trace=False,
                 stats=False, p=0, graph=True, tune=None, perc=100, rough_fix=False):
    """Options plus the Python objects that must stay alive during the call.
    trace: False, True (every iteration), a set of iterations to keep, or a
    callable that receives each iteration's record (nothing is kept).
    perc / rough_fix: the two options outside Algorithm 1 (boruta_options)."""
    o = boruta_default_options()
    o.n_bins, o.n_perm, o.split_rank, o.form = n_bins, n_perm, split_rank, form
    o.graph = int(bool(graph))
    o.perc, o.rough_fix = int(perc), int(bool(rough_fix))
    for k, v in (tune or {}).items():
        if k == "tune_cache":  # a path (see include/boruta.h)
            keep_cache = str(v).encode()
            o.tune_cache = keep_cache
            continue
        if k not in TUNE_KEYS:
            raise ValueError(f"unknown tuning key {k}")
        setattr(o, k, int(v))
    keep = {"iters": [], "cache_path": o.tune_cache}
    if callable(trace):
        keep["sink"] = trace
        keep["cb"] = _trace_collector(keep, p, None)
        o.trace = keep["cb"]
    elif trace is not False:
        keep["cb"] = _trace_collector(keep, p, None if trace is True else set(trace))
        o.trace = keep["cb"]
    if stats:
        keep["stats"] = Stats()
        o.stats = ctypes.pointer(keep["stats"])
    return o, keep


def boruta_fit_ex(X, y, n_classes, n_trees, max_depth, mtry=0, importance_mode=TREEIMP,
                  max_iter=20, alpha=0.05, seed=0, n_bins=256, n_perm=1, split_rank=RANK_FP32,
                  form=FORM_BATCHED, trace=False, stats=False, graph=True, tune=None, perc=100,
                  rough_fix=False):
    """Host arrays in, host arrays out (see boruta_fit in include/boruta.h)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n, p = X.shape
    dec = np.zeros(p, np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = np.zeros(1, np.int32)
    o, keep = make_options(n_bins, n_perm, split_rank, form, trace, stats, p, graph, tune, perc,
                           rough_fix)
    rc = lib().boruta_fit_ex(_ptr(X), _ptr(y), n, p, n_classes, n_trees, max_depth, mtry,
                             importance_mode, max_iter, alpha, seed, ctypes.byref(o), _ptr(dec),
                             _ptr(hist), _ptr(hits), _ptr(smax), _ptr(n_iter))
    _check(rc)
    out = {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
           "n_iter": int(n_iter[0]), "traces": keep["iters"]}
    if stats:
        out["stats"] = keep["stats"]
    return out


def boruta_fit_regression(X, y, n_trees, max_depth, mtry=0, importance_mode=TREEIMP,
                          max_iter=20, alpha=0.05, seed=0, n_bins=256, n_perm=1,
                          split_rank=RANK_FP32,
                          form=FORM_BATCHED, trace=False, stats=False, graph=True, tune=None,
                          perc=100, rough_fix=False):
    """Regression Boruta: y float targets (see boruta_fit_regression in
    include/boruta.h)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n, p = X.shape
    dec = np.zeros(p, np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = np.zeros(1, np.int32)
    o, keep = make_options(n_bins, n_perm, split_rank, form, trace, stats, p, graph, tune, perc,
                           rough_fix)
    rc = lib().boruta_fit_regression(_ptr(X), _ptr(y), n, p, n_trees, max_depth, mtry,
                                     importance_mode, max_iter, alpha, seed, ctypes.byref(o),
                                     _ptr(dec), _ptr(hist), _ptr(hits), _ptr(smax), _ptr(n_iter))
    _check(rc)
    out = {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
           "n_iter": int(n_iter[0]), "traces": keep["iters"]}
    if stats:
        out["stats"] = keep["stats"]
    return out


def boruta_fit(X, y, n_classes, n_trees, max_depth, mtry=0, importance_mode=TREEIMP,
               max_iter=20, alpha=0.05, seed=0):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n, p = X.shape
    dec = np.zeros(p, np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = np.zeros(1, np.int32)
    rc = lib().boruta_fit(_ptr(X), _ptr(y), n, p, n_classes, n_trees, max_depth, mtry,
                          importance_mode, max_iter, alpha, seed, _ptr(dec), _ptr(hist),
                          _ptr(hits), _ptr(smax), _ptr(n_iter))
    _check(rc)
    return {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
            "n_iter": int(n_iter[0])}


def _job(X, y, n_classes, n_trees, max_depth, mtry, importance_mode, max_iter, alpha, seed):
    j = Job()
    j.X, j.y = X.ctypes.data, y.ctypes.data
    j.n, j.p = X.shape
    j.n_classes, j.n_trees, j.max_depth, j.mtry = n_classes, n_trees, max_depth, mtry
    j.importance_mode, j.max_iter, j.alpha, j.seed = importance_mode, max_iter, alpha, seed
    return j


def boruta_fit_batch(jobs, n_bins=256, n_perm=1, split_rank=RANK_FP32, form=FORM_BATCHED,
                     trace=False, stats=False, perc=100, rough_fix=False, tune=None):
    """jobs: list of dicts with X, y, n_classes, n_trees, max_depth and optional mtry,
    importance_mode, max_iter, alpha, seed; a regression job has y_reg (float
    targets) instead of y and n_classes.  tune: launch-shape fields as for
    boruta_fit_ex."""
    arrs, cj, res, outs = [], (Job * len(jobs))(), (Result * len(jobs))(), []
    for i, jd in enumerate(jobs):
        X = np.ascontiguousarray(jd["X"], dtype=np.float32)
        yr = None
        if jd.get("y_reg") is not None:
            yr = np.ascontiguousarray(jd["y_reg"], dtype=np.float32)
            y = np.zeros(1, np.int32)
        else:
            y = np.ascontiguousarray(jd["y"], dtype=np.int32)
        max_iter = jd.get("max_iter", 20)
        p = X.shape[1]
        cj[i] = _job(X, y, jd.get("n_classes", 2), jd["n_trees"], jd["max_depth"],
                     jd.get("mtry", 0), jd.get("importance_mode", TREEIMP), max_iter,
                     jd.get("alpha", 0.05), jd.get("seed", 0))
        if yr is not None:
            cj[i].y_reg = yr.ctypes.data
        o = {"decision": np.zeros(p, np.int8), "imp_history": np.full((max_iter, p), np.nan),
             "hits": np.zeros(p, np.int32), "shadow_max": np.full(max_iter, np.nan),
             "rank": np.zeros(p, np.int32)}
        res[i].decision = o["decision"].ctypes.data
        res[i].imp_history = o["imp_history"].ctypes.data
        res[i].hits = o["hits"].ctypes.data
        res[i].shadow_max = o["shadow_max"].ctypes.data
        res[i].rank = o["rank"].ctypes.data
        arrs.append((X, y, yr))
        outs.append(o)
    p_all = [int(np.shape(jd["X"])[1]) for jd in jobs]
    opt, keep = make_options(n_bins, n_perm, split_rank, form, trace, stats, p_all,
                             tune=tune, perc=perc, rough_fix=rough_fix)
    rc = lib().boruta_fit_batch(cj, len(jobs), ctypes.byref(opt), res)
    for i, o in enumerate(outs):
        o["n_iter"], o["status"] = res[i].n_iter, res[i].status
    _check(rc)
    return {"results": outs, "traces": keep["iters"], "stats": keep.get("stats")}


def boruta_fit_seeds(X, y, n_classes, n_trees, max_depth, seeds, mtry=0,
                     importance_mode=TREEIMP, max_iter=20, alpha=0.05, n_bins=256, n_perm=1,
                     split_rank=RANK_FP32, form=FORM_BATCHED, tune=None, runs=True, perc=100,
                     rough_fix=False):
    """One problem run once per seed (as one batch) and the multi-seed aggregate:
    returns {"median_importance", "decision", "runs"} where runs (if asked for)
    holds each seed's own results as boruta_fit_batch does.  n_classes=None:
    a regression problem with float targets y."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    regression = n_classes is None
    y = np.ascontiguousarray(y, dtype=np.float32 if regression else np.int32)
    n, p = X.shape
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    med = np.zeros(p, np.float64)
    dec = np.zeros(p, np.int8)
    res, outs = None, []
    if runs:
        res = (Result * len(sd))()
        for i in range(len(sd)):
            o = {"decision": np.zeros(p, np.int8),
                 "imp_history": np.full((max_iter, p), np.nan),
                 "hits": np.zeros(p, np.int32), "shadow_max": np.full(max_iter, np.nan),
                 "rank": np.zeros(p, np.int32)}
            res[i].decision = o["decision"].ctypes.data
            res[i].imp_history = o["imp_history"].ctypes.data
            res[i].hits = o["hits"].ctypes.data
            res[i].shadow_max = o["shadow_max"].ctypes.data
            res[i].rank = o["rank"].ctypes.data
            outs.append(o)
    opt, _ = make_options(n_bins, n_perm, split_rank, form, tune=tune, perc=perc,
                          rough_fix=rough_fix)
    if regression:
        rc = lib().boruta_fit_seeds_regression(_ptr(X), _ptr(y), n, p, n_trees, max_depth, mtry,
                                               importance_mode, max_iter, alpha, _ptr(sd),
                                               len(sd), ctypes.byref(opt), _ptr(med), _ptr(dec),
                                               res)
    else:
        rc = lib().boruta_fit_seeds(_ptr(X), _ptr(y), n, p, n_classes, n_trees, max_depth, mtry,
                                    importance_mode, max_iter, alpha, _ptr(sd), len(sd),
                                    ctypes.byref(opt), _ptr(med), _ptr(dec), res)
    for i, o in enumerate(outs):
        o["n_iter"], o["status"] = res[i].n_iter, res[i].status
    _check(rc)
    return {"median_importance": med, "decision": dec, "runs": outs}


def boruta_workspace_size(jobs, n_bins=256, n_perm=1, split_rank=RANK_FP32,
                          form=FORM_BATCHED, tune=None):
    """jobs: list of dicts with shapes (X may be any array with .shape)."""
    cj = (Job * len(jobs))()
    for i, jd in enumerate(jobs):
        j = Job()
        j.X, j.y = 1, 1
        j.n, j.p = jd["n"], jd["p"]
        j.n_classes, j.n_trees, j.max_depth = jd.get("n_classes", 2), jd["n_trees"], \
            jd["max_depth"]
        j.mtry, j.importance_mode = jd.get("mtry", 0), jd.get("importance_mode", TREEIMP)
        j.max_iter, j.alpha, j.seed = jd.get("max_iter", 20), jd.get("alpha", 0.05), 0
        if jd.get("regression"):
            j.y_reg = 1
        cj[i] = j
    opt, _ = make_options(n_bins, n_perm, split_rank, form, tune=tune)
    out = ctypes.c_size_t(0)
    _check(lib().boruta_workspace_size(cj, len(jobs), ctypes.byref(opt), ctypes.byref(out)))
    return int(out.value)


def boruta_fit_device(dX, dy, n_classes, n_trees, max_depth, workspace, stream=None, mtry=0,
                      importance_mode=TREEIMP, max_iter=20, alpha=0.05, seed=0, n_bins=256,
                      n_perm=1, split_rank=RANK_FP32, form=FORM_BATCHED, trace=False,
                      stats=False, perc=100, rough_fix=False):
    """dX [n][p] float32, dy [n] int32 and workspace (uint8) are torch CUDA tensors; stream a
    torch.cuda.Stream (default: the current stream)."""
    import torch
    assert dX.is_cuda and dy.is_cuda and workspace.is_cuda
    assert dX.dtype == torch.float32 and dy.dtype == torch.int32 and dX.is_contiguous()
    n, p = dX.shape
    st = stream if stream is not None else torch.cuda.current_stream(dX.device)
    dec = np.zeros(p, np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = np.zeros(1, np.int32)
    opt, keep = make_options(n_bins, n_perm, split_rank, form, trace, stats, p, perc=perc,
                             rough_fix=rough_fix)
    rc = lib().boruta_fit_device(dX.data_ptr(), dy.data_ptr(), n, p, n_classes, n_trees,
                                 max_depth, mtry, importance_mode, max_iter, alpha, seed,
                                 ctypes.byref(opt), workspace.data_ptr(), workspace.numel(),
                                 st.cuda_stream, _ptr(dec), _ptr(hist), _ptr(hits), _ptr(smax),
                                 _ptr(n_iter))
    _check(rc)
    out = {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
           "n_iter": int(n_iter[0]), "traces": keep["iters"]}
    if stats:
        out["stats"] = keep["stats"]
    return out


def boruta_fit_device_noalloc(dX, dy, n_classes, n_trees, max_depth, stream=None, mtry=0,
                              importance_mode=TREEIMP, max_iter=20, alpha=0.05, seed=0,
                              n_bins=256, n_perm=1, split_rank=RANK_FP32, perc=100,
                              rough_fix=False):
    """boruta_fit_device without a workspace: the library's static device
    scratch serves (see include/boruta.h).  dX [n][p] float32 and dy [n] int32
    are contiguous torch CUDA tensors."""
    import torch
    _check_device_input(dX, "float32", 2, "X")
    _check_device_input(dy, "int32", 1, "y")
    n, p = dX.shape
    st = stream if stream is not None else torch.cuda.current_stream(dX.device)
    dec = np.zeros(p, np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = np.zeros(1, np.int32)
    opt, _ = make_options(n_bins, n_perm, split_rank, FORM_BATCHED, False, False, p, perc=perc,
                          rough_fix=rough_fix)
    rc = lib().boruta_fit_device_noalloc(dX.data_ptr(), dy.data_ptr(), n, p, n_classes,
                                         n_trees, max_depth, mtry, importance_mode, max_iter,
                                         alpha, seed, ctypes.byref(opt), st.cuda_stream,
                                         _ptr(dec), _ptr(hist), _ptr(hits), _ptr(smax),
                                         _ptr(n_iter))
    _check(rc)
    return {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
            "n_iter": int(n_iter[0])}


def boruta_bin(X, n_bins=256):
    """Quantile bins of X [n][p] computed on the device: uint8 [p][n]."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, p = X.shape
    out = np.zeros((p, n), np.uint8)
    _check(lib().boruta_bin(_ptr(X), n, p, n_bins, _ptr(out)))
    return out


def boruta_probe_copy(dst, src, nbytes, stream=None):
    """Device-to-device streaming copy of torch tensors (counter calibration)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(dst.device)
    _check(lib().boruta_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream))


def _check_device_input(t, dtype, ndim, name):
    """A device input is handed over as a raw pointer: it must be a contiguous
    CUDA tensor of the stated dtype and rank (a strided view would be read
    as if it were row-major)."""
    if not (getattr(t, "is_cuda", False) and str(t.dtype) == "torch." + dtype and
            t.dim() == ndim and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of rank {ndim}")


class Session:
    """boruta_session_* wrapper.  jobs as for boruta_fit_batch; with
    inputs_on_device, X/y are torch CUDA tensors (float32 [n][p], int32 [n])."""

    def __init__(self, jobs, n_bins=256, n_perm=1, split_rank=RANK_FP32, form=FORM_BATCHED,
                 trace=False, stats=False, inputs_on_device=False, workspace=None, stream=None,
                 graph=True, tune=None, perc=100, rough_fix=False):
        self._arrays, cj = [], (Job * len(jobs))()
        self._shapes = []
        for i, jd in enumerate(jobs):
            yr, rp = jd.get("y_reg"), None
            if inputs_on_device:
                X, y = jd["X"], jd.get("y")
                _check_device_input(X, "float32", 2, "X")
                if y is not None:
                    _check_device_input(y, "int32", 1, "y")
                if yr is not None:
                    _check_device_input(yr, "float32", 1, "y_reg")
                xp = X.data_ptr()
                yp = y.data_ptr() if y is not None else None
                rp = yr.data_ptr() if yr is not None else None
                n, p = X.shape
            else:
                X = np.ascontiguousarray(jd["X"], dtype=np.float32)
                y = np.ascontiguousarray(jd["y"], dtype=np.int32) if yr is None else None
                if yr is not None:
                    yr = np.ascontiguousarray(yr, dtype=np.float32)
                    rp = yr.ctypes.data
                xp, yp = X.ctypes.data, (y.ctypes.data if y is not None else None)
                n, p = X.shape
            self._arrays.append((X, y, yr))
            j = Job()
            j.X, j.y, j.n, j.p = xp, yp, n, p
            j.y_reg = rp
            j.n_classes = jd.get("n_classes", 2)
            j.n_trees, j.max_depth = jd["n_trees"], jd["max_depth"]
            j.mtry, j.importance_mode = jd.get("mtry", 0), jd.get("importance_mode", TREEIMP)
            j.max_iter, j.alpha, j.seed = jd.get("max_iter", 20), jd.get("alpha", 0.05), \
                jd.get("seed", 0)
            cj[i] = j
            self._shapes.append((p, j.max_iter))
        p_all = [int(sh[0]) for sh in self._shapes]
        self.opt, self.keep = make_options(n_bins, n_perm, split_rank, form, trace, stats, p_all,
                                           graph, tune, perc, rough_fix)
        self._jobs = cj
        self._ws = workspace
        ws_ptr = workspace.data_ptr() if workspace is not None else None
        ws_len = workspace.numel() if workspace is not None else 0
        st = None
        if stream is not None:
            st = stream.cuda_stream
        h = ctypes.c_void_p()
        _check(lib().boruta_session_create(cj, len(jobs), ctypes.byref(self.opt),
                                           int(inputs_on_device), ws_ptr, ws_len, st,
                                           ctypes.byref(h)))
        self.h = h

    @property
    def stats(self):
        return self.keep.get("stats")

    @property
    def traces(self):
        return self.keep["iters"]

    def step(self):
        n = ctypes.c_int32(0)
        _check(lib().boruta_session_step(self.h, ctypes.byref(n)))
        return n.value

    def run(self, max_steps):
        """Up to max_steps iterations enqueued back to back; returns (jobs
        still live, job-iterations run)."""
        n, done = ctypes.c_int32(0), ctypes.c_int64(0)
        _check(lib().boruta_session_run(self.h, max_steps, ctypes.byref(n), ctypes.byref(done)))
        return n.value, done.value

    def result(self, job=0):
        p, max_iter = self._shapes[job]
        o = {"decision": np.zeros(p, np.int8), "imp_history": np.full((max_iter, p), np.nan),
             "hits": np.zeros(p, np.int32), "shadow_max": np.full(max_iter, np.nan),
             "rank": np.zeros(p, np.int32)}
        r = Result()
        r.decision = o["decision"].ctypes.data
        r.imp_history = o["imp_history"].ctypes.data
        r.hits = o["hits"].ctypes.data
        r.shadow_max = o["shadow_max"].ctypes.data
        r.rank = o["rank"].ctypes.data
        _check(lib().boruta_session_result(self.h, job, ctypes.byref(r)))
        o["n_iter"] = r.n_iter
        return o

    def resume(self, job, t, state, hits):
        st = np.ascontiguousarray(state, dtype=np.int8)
        ht = np.ascontiguousarray(hits, dtype=np.int32)
        _check(lib().boruta_session_resume(self.h, job, t, _ptr(st), _ptr(ht)))

    def close(self):
        if getattr(self, "h", None):
            lib().boruta_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
