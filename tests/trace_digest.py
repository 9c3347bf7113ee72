"""Digests of per-iteration trace records and of finished runs, so that whole
runs can be compared with stored oracle results without keeping every tree.

A record digest is the SHA-256 of the record's integers in a fixed order
(iteration, widths, then the widened-column sources, integer importances,
hits, states, per-tree statistics and the node table), each as little-endian
int64.  Both sides' records hold exactly these integers, so equal digests
mean equal records.
"""
import hashlib

import numpy as np

FIELDS = ("col_src", "imp_int", "hits", "state", "tree_stats", "nodes")


def record_digest(rec):
    h = hashlib.sha256()
    head = np.array([rec["t"], rec["p_cur"], rec["n_sha"], rec["p_w"], rec["mtry"]], np.int64)
    h.update(head.tobytes())
    for k in FIELDS:
        a = np.ascontiguousarray(np.asarray(rec[k]).astype(np.int64, copy=False))
        h.update(np.array([a.size], np.int64).tobytes())
        h.update(a.astype("<i8", copy=False).tobytes())
    return h.hexdigest()


def record_summary(rec):
    """A few readable figures of a record (for messages when digests differ)."""
    nodes = np.asarray(rec["nodes"])
    return {"t": int(rec["t"]), "p_w": int(rec["p_w"]), "mtry": int(rec["mtry"]),
            "n_nodes": int(nodes.shape[0]),
            "n_split": int((nodes[:, 2] >= 0).sum()) if nodes.size else 0,
            "imp_sum": int(np.asarray(rec["imp_int"], np.int64).sum()),
            "hits_sum": int(np.asarray(rec["hits"], np.int64).sum())}


class Digester:
    """Trace sink: keeps one (digest, summary) per record, per job."""

    def __init__(self):
        self.by_job = {}

    def __call__(self, rec):
        self.by_job.setdefault(int(rec.get("job", 0)), []).append(
            {"digest": record_digest(rec), **record_summary(rec)})


def history_digest(hist, n_iter):
    """SHA-256 of the first n_iter rows of an importance history (IEEE double
    bytes, NaN entries written as one canonical NaN)."""
    a = np.array(hist[:n_iter], dtype="<f8", copy=True)
    a[np.isnan(a)] = np.nan
    return hashlib.sha256(a.tobytes()).hexdigest()


def run_summary(r):
    """The final outputs of a run: decisions, hits, rank, iterations, and
    digests of the history and the per-iteration shadow maxima."""
    k = int(r["n_iter"])
    return {"n_iter": k,
            "decision": np.asarray(r["decision"], np.int64).tolist(),
            "hits": np.asarray(r["hits"], np.int64).tolist(),
            "rank": np.asarray(r["rank"], np.int64).tolist(),
            "history_sha256": history_digest(r["imp_history"], k),
            "shadow_max_sha256": history_digest(np.asarray(r["shadow_max"])[:, None], k)}
