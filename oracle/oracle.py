"""TEST INFRASTRUCTURE ONLY: ctypes bindings to the CPU oracle.

The oracle (``boruta_oracle.cpp``) is a plain, slow CPU reference of one
Boruta run (Algorithm 1; impurity importance of Algorithm 2, Sec. 2.1;
out-of-bag permutation importance, Sec. 2 and 2.2; the prediction-divergence
permutation importance of Algorithm 3, Sec. 2.2).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this module.
It shares no code with the HIP library.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "boruta_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_boruta.so")

STREAM_BOOT, STREAM_MTRY, STREAM_SHADOW, STREAM_OOBPERM, STREAM_FLUSH = 1, 2, 3, 4, 5


def build():
    """Compile the oracle with g++ (plain C++17, no fused multiply-add)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
           "-pthread", SRC, "-o", LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)


class IterTrace(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int32), ("p_cur", ctypes.c_int32), ("n_sha", ctypes.c_int32),
        ("p_w", ctypes.c_int32), ("mtry", ctypes.c_int32), ("n_trees", ctypes.c_int32),
        ("col_src", ctypes.POINTER(ctypes.c_int32)),
        ("imp_int", ctypes.POINTER(ctypes.c_int64)),
        ("hits", ctypes.POINTER(ctypes.c_int32)),
        ("state", ctypes.POINTER(ctypes.c_int8)),
        ("tree_stats", ctypes.POINTER(ctypes.c_int64)),
        ("n_nodes", ctypes.c_int64),
        ("nodes", ctypes.POINTER(ctypes.c_int64)),
    ]


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(IterTrace))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_keyed_perm.argtypes = [u64, u32, u32, u32, u32, u32, u64, u64]
        L.oracle_keyed_perm.restype = u64
        L.oracle_bin.argtypes = [P, i64, i64, i32, P, P, P]
        L.oracle_bin.restype = i32
        L.oracle_log2_fix32.argtypes = [u64]
        L.oracle_log2_fix32.restype = u64
        L.oracle_kl_fix32.argtypes = [P, P, i32]
        L.oracle_kl_fix32.restype = i64
        L.oracle_seed_median.argtypes = [P, P, P, i64, i32, i32, P, P]
        L.oracle_seed_median.restype = None
        L.oracle_rank.argtypes = [P, P, i64, i32, P]
        L.oracle_rank.restype = None
        L.oracle_bootstrap.argtypes = [u64, u32, u32, i64, P]
        L.oracle_bootstrap.restype = None
        L.oracle_best_split.argtypes = [P, i64, P, P, P, i64, P, i32, i32, i32, P]
        L.oracle_best_split.restype = i32
        L.oracle_grow_tree.argtypes = [P, i64, i64, P, P, i32, i32, i32, i32, u64, u32, u32,
                                       P, i64, P]
        L.oracle_grow_tree.restype = i64
        L.oracle_binom_decide.argtypes = [i32, i32, i64, f64]
        L.oracle_binom_decide.restype = i32
        L.oracle_boruta_fit.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, i32, f64, u64,
                                        i32, i32, i32, i32, P, P, P, P, P, TRACE_FN, P]
        L.oracle_boruta_fit.restype = i32
        L.oracle_boruta_fit_ext.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, i32, f64,
                                            u64, i32, i32, i32, i32, i32, i32, P, P, P, P, P,
                                            TRACE_FN, P]
        L.oracle_boruta_fit_ext.restype = i32
        L.oracle_boruta_fit_reg.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, f64, u64,
                                            i32, i32, i32, i32, P, P, P, P, P, TRACE_FN, P]
        L.oracle_boruta_fit_reg.restype = i32
        L.oracle_fix_targets.argtypes = [P, i64, i32, i32, P, P]
        L.oracle_fix_targets.restype = i32
        L.oracle_best_split_reg.argtypes = [P, i64, P, P, P, i64, P, i32, i32, i32, P]
        L.oracle_best_split_reg.restype = i32
        L.oracle_shadow_threshold.argtypes = [P, i32, i32]
        L.oracle_shadow_threshold.restype = i64
        L.oracle_rough_fix.argtypes = [P, P, P, i64, i32]
        L.oracle_rough_fix.restype = None
        L.oracle_boruta_step.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, f64, u64, i32,
                                         i32, i32, P, P, P, i32, i32, i32, P, P, TRACE_FN, P]
        L.oracle_boruta_step.restype = i32
        L.oracle_boruta_step_cols.argtypes = [P, P, i64, i64, i32, i32, i32, i32, i32, f64, u64,
                                              i32, i32, i32, P, P, P, i32, P, i32, i32, i32, P, P,
                                              TRACE_FN, P]
        L.oracle_boruta_step_cols.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def keyed_perm(seed, stream, t, a, b, c_hi, m, x):
    return int(lib().oracle_keyed_perm(seed, stream, t, a, b, c_hi, m, x))


def bin_matrix(X, n_bins):
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, p = X.shape
    bins = np.zeros((p, n), dtype=np.uint8)
    cuts = np.zeros((p, n_bins - 1), dtype=np.float32)
    ncuts = np.zeros(p, dtype=np.int32)
    rc = lib().oracle_bin(_ptr(X), n, p, n_bins, _ptr(bins), _ptr(cuts), _ptr(ncuts))
    if rc:
        raise ValueError(f"oracle_bin failed: {rc}")
    return bins, cuts, ncuts


def log2_fix32(x):
    return int(lib().oracle_log2_fix32(int(x)))


def kl_fix32(S, Sq):
    S = np.ascontiguousarray(S, dtype=np.uint64)
    Sq = np.ascontiguousarray(Sq, dtype=np.uint64)
    return int(lib().oracle_kl_fix32(_ptr(S), _ptr(Sq), len(S)))


def bootstrap(seed, t, tree, n):
    w = np.zeros(n, dtype=np.uint32)
    lib().oracle_bootstrap(seed, t, tree, n, _ptr(w))
    return w


def best_split(bins, y, w, rows, feats, n_classes, n_bins):
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    feats = np.ascontiguousarray(feats, dtype=np.int32)
    out = np.zeros(8, dtype=np.uint64)
    rc = lib().oracle_best_split(_ptr(bins), bins.shape[1], _ptr(y), _ptr(w), _ptr(rows),
                                 len(rows), _ptr(feats), len(feats), n_classes, n_bins, _ptr(out))
    if rc:
        raise ValueError("oracle_best_split failed")
    keys = ["found", "q", "b", "nl", "sl", "nr", "sr", "gain_fix"]
    return {k: int(v) for k, v in zip(keys, out)}


def best_split_reg(bins, yfix, w, rows, feats, n_bins, s_gain=0):
    """Best regression split of one node with fixed-point targets yfix (int64):
    found, draw position q, bin b, W_L (wl), W_R (wr), T_L (tl), T_R (tr) and
    floor(D / 2^s_gain)."""
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    yfix = np.ascontiguousarray(yfix, dtype=np.int64)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    feats = np.ascontiguousarray(feats, dtype=np.int32)
    out = np.zeros(8, dtype=np.int64)
    rc = lib().oracle_best_split_reg(_ptr(bins), bins.shape[1], _ptr(yfix), _ptr(w), _ptr(rows),
                                     len(rows), _ptr(feats), len(feats), n_bins, s_gain,
                                     _ptr(out))
    if rc:
        raise ValueError("oracle_best_split_reg failed")
    keys = ["found", "q", "b", "wl", "wr", "tl", "tr", "gain_fix"]
    return {k: int(v) for k, v in zip(keys, out)}


def fix_targets(y, n_trees=1, n_perm=1):
    """Fixed-point targets of float32 y: (y_fix int64, e, shifts) with
    y_fix = rint(y 2^(38 - e)) and shifts = dict(s_gain, s_perm, s_kl, range)."""
    y = np.ascontiguousarray(y, dtype=np.float32)
    out = np.zeros(y.shape[0], dtype=np.int64)
    sh = np.zeros(4, dtype=np.int64)
    e = lib().oracle_fix_targets(_ptr(y), y.shape[0], n_trees, n_perm, _ptr(out), _ptr(sh))
    return out, int(e), dict(zip(("s_gain", "s_perm", "s_kl", "range"), map(int, sh)))


def grow_tree(bins, y, w, n_classes, n_bins, max_depth, mtry, seed, t, tree):
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    p_w, n = bins.shape
    y = np.ascontiguousarray(y, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    cap = 2 * n + 2
    nodes = np.zeros((cap, 6), dtype=np.int64)
    gains = np.zeros(p_w, dtype=np.uint64)
    cnt = lib().oracle_grow_tree(_ptr(bins), n, p_w, _ptr(y), _ptr(w), n_classes, n_bins,
                                 max_depth, mtry, seed, t, tree, _ptr(nodes), cap, _ptr(gains))
    if cnt < 0:
        raise ValueError("oracle_grow_tree failed")
    return nodes[:cnt].copy(), gains


def binom_decide(hits, t, p, alpha):
    return int(lib().oracle_binom_decide(hits, t, p, alpha))


def _trace_collector(store, p=None):
    """Copies each iteration record into the list `store`, or, when `store`
    is a callable, hands the record to it (and keeps nothing).  p: the
    feature count (hits and state are copied when given)."""
    def cb(_user, trp):
        tr = trp.contents
        p_w, nt, nn = tr.p_w, tr.n_trees, tr.n_nodes
        rec = {
            "t": tr.t, "p_cur": tr.p_cur, "n_sha": tr.n_sha, "p_w": p_w, "mtry": tr.mtry,
            "col_src": np.ctypeslib.as_array(tr.col_src, (p_w,)).copy(),
            "imp_int": np.ctypeslib.as_array(tr.imp_int, (p_w,)).copy(),
            "tree_stats": np.ctypeslib.as_array(tr.tree_stats, (nt, 5)).copy() if nt else
            np.zeros((0, 5), np.int64),
            "nodes": np.ctypeslib.as_array(tr.nodes, (nn, 6)).copy() if nn else
            np.zeros((0, 6), np.int64),
        }
        if p is not None:
            rec["hits"] = np.ctypeslib.as_array(tr.hits, (p,)).copy()
            rec["state"] = np.ctypeslib.as_array(tr.state, (p,)).copy()
        if callable(store):
            store(rec)
        else:
            store.append(rec)
    return TRACE_FN(cb)


def _collector_for(trace, traces, p):
    """trace: False, True (records kept in `traces`) or a callable."""
    if callable(trace):
        return _trace_collector(trace, p)
    return _trace_collector(traces, p) if trace else TRACE_FN()


def boruta_fit(X, y, n_classes, n_trees, max_depth, mtry=0, importance_mode=0, max_iter=20,
               alpha=0.05, seed=0, n_bins=256, n_perm=1, n_threads=0, permut_naive=False,
               trace=False, perc=100, rough_fix=False):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n, p = X.shape
    dec = np.zeros(p, dtype=np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, dtype=np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = ctypes.c_int32(0)
    traces = []
    cb = _collector_for(trace, traces, p)
    rc = lib().oracle_boruta_fit_ext(_ptr(X), _ptr(y), n, p, n_classes, n_trees, max_depth,
                                     mtry, importance_mode, max_iter, alpha, seed, n_bins,
                                     n_perm, n_threads, int(permut_naive), perc,
                                     int(bool(rough_fix)), _ptr(dec), _ptr(hist), _ptr(hits),
                                     _ptr(smax),
                                     ctypes.cast(ctypes.byref(n_iter), ctypes.c_void_p), cb,
                                     None)
    if rc:
        raise ValueError(f"oracle_boruta_fit failed: {rc}")
    rank = np.zeros(p, dtype=np.int32)
    hist_c = np.ascontiguousarray(hist)
    lib().oracle_rank(_ptr(dec), _ptr(hist_c), p, n_iter.value, _ptr(rank))
    return {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
            "n_iter": n_iter.value, "traces": traces, "rc": rc, "rank": rank}


def boruta_fit_reg(X, y, n_trees, max_depth, mtry=0, importance_mode=0, max_iter=20,
                   alpha=0.05, seed=0, n_bins=256, n_perm=1, n_threads=0, permut_naive=False,
                   trace=False):
    """Regression Boruta (TreeImp or Permut): y float targets."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n, p = X.shape
    dec = np.zeros(p, dtype=np.int8)
    hist = np.full((max_iter, p), np.nan)
    hits = np.zeros(p, dtype=np.int32)
    smax = np.full(max_iter, np.nan)
    n_iter = ctypes.c_int32(0)
    traces = []
    cb = _collector_for(trace, traces, p)
    rc = lib().oracle_boruta_fit_reg(_ptr(X), _ptr(y), n, p, n_trees, max_depth, mtry,
                                     importance_mode, max_iter, alpha, seed, n_bins, n_perm,
                                     n_threads, int(permut_naive),
                                     _ptr(dec), _ptr(hist), _ptr(hits), _ptr(smax),
                                     ctypes.cast(ctypes.byref(n_iter), ctypes.c_void_p), cb,
                                     None)
    if rc:
        raise ValueError(f"oracle_boruta_fit_reg failed: {rc}")
    rank = np.zeros(p, dtype=np.int32)
    lib().oracle_rank(_ptr(dec), _ptr(np.ascontiguousarray(hist)), p, n_iter.value, _ptr(rank))
    return {"decision": dec, "imp_history": hist, "hits": hits, "shadow_max": smax,
            "n_iter": n_iter.value, "traces": traces, "rc": rc, "rank": rank}


def shadow_threshold(sha, perc):
    """Hit threshold over shadow importances (integers) at percentile perc."""
    a = np.ascontiguousarray(sha, dtype=np.int64)
    return int(lib().oracle_shadow_threshold(_ptr(a), a.shape[0], perc))


def rough_fix(decision, imp_history, shadow_max, n_iter):
    """Rough fix of the tentative features of a finished run (a new array)."""
    dec = np.array(decision, dtype=np.int8)
    hist = np.ascontiguousarray(imp_history, dtype=np.float64)
    smax = np.ascontiguousarray(shadow_max, dtype=np.float64)
    lib().oracle_rough_fix(_ptr(dec), _ptr(hist), _ptr(smax), dec.shape[0], n_iter)
    return dec


def seed_median(runs):
    """Multi-seed aggregate of finished runs (dicts of boruta_fit): per feature
    the median of the runs' mean history importances and the lower median of
    their decisions."""
    dec = np.ascontiguousarray(np.stack([r["decision"] for r in runs]), dtype=np.int8)
    hist = np.ascontiguousarray(np.stack([r["imp_history"] for r in runs]), dtype=np.float64)
    n_it = np.ascontiguousarray([r["n_iter"] for r in runs], dtype=np.int32)
    n_runs, max_iter, p = hist.shape
    med = np.zeros(p, np.float64)
    out = np.zeros(p, np.int8)
    lib().oracle_seed_median(_ptr(dec), _ptr(hist), _ptr(n_it), p, max_iter, n_runs, _ptr(med),
                             _ptr(out))
    return med, out


def rank(decision, imp_history, n_iter):
    dec = np.ascontiguousarray(decision, dtype=np.int8)
    hist = np.ascontiguousarray(imp_history, dtype=np.float64)
    out = np.zeros(dec.shape[0], dtype=np.int32)
    lib().oracle_rank(_ptr(dec), _ptr(hist), dec.shape[0], n_iter, _ptr(out))
    return out


def boruta_step(X, y, n_classes, n_trees, max_depth, t, state, hits, mtry=0,
                importance_mode=0, alpha=0.05, seed=0, n_bins=256, n_perm=1, tree_subset=None,
                n_threads=0, permut_naive=False, trace=True, kl_cols=None):
    """Iteration t of Algorithm 1 from the given (state, hits); returns the
    updated vectors, the importance row and the trace record.  kl_cols (mode
    2): score only these widened columns (the others read 0)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n, p = X.shape
    st = np.array(state, dtype=np.int8, copy=True)
    ht = np.array(hits, dtype=np.int32, copy=True)
    row = np.full(p, np.nan)
    smax = np.zeros(1)
    sub = None if tree_subset is None else np.ascontiguousarray(tree_subset, dtype=np.int32)
    n_sub = 0 if sub is None else len(sub)
    if sub is not None and n_sub == 0:
        sub = np.zeros(1, np.int32)  # non-null pointer, zero trees: widening only
    traces = []
    cb = _collector_for(trace, traces, p)
    kc = None if kl_cols is None else np.ascontiguousarray(kl_cols, dtype=np.int32)
    rc = lib().oracle_boruta_step_cols(_ptr(X), _ptr(y), n, p, n_classes, n_trees, max_depth,
                                       mtry, importance_mode, alpha, seed, n_bins, n_perm, t,
                                       _ptr(st), _ptr(ht), _ptr(sub), n_sub, _ptr(kc),
                                       0 if kc is None else len(kc), n_threads,
                                       int(permut_naive), _ptr(row), _ptr(smax), cb, None)
    if rc:
        raise ValueError(f"oracle_boruta_step failed: {rc}")
    return {"state": st, "hits": ht, "imp_row": row, "shadow_max": float(smax[0]),
            "trace": traces[0] if traces else None}
