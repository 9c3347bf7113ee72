"""Comparison of a HIP run with the CPU oracle: integers and decisions
bit-exact, reported importances exactly equal (both sides divide the same
exact integers once in IEEE double precision)."""
import numpy as np


def assert_same_trace(g, o, trees=None):
    assert g["t"] == o["t"]
    assert (g["p_cur"], g["n_sha"], g["p_w"], g["mtry"]) == \
        (o["p_cur"], o["n_sha"], o["p_w"], o["mtry"])
    assert np.array_equal(g["col_src"], o["col_src"])
    gn, on = g["nodes"], o["nodes"]
    gs, os_ = g["tree_stats"], o["tree_stats"]
    if trees is not None:
        gn = gn[np.isin(gn[:, 0], trees)]
        gs = gs[np.isin(gs[:, 0], trees)]
    else:
        assert np.array_equal(g["imp_int"], o["imp_int"])
    assert gn.shape == on.shape, (gn.shape, on.shape)
    bad = np.flatnonzero(np.any(gn != on, axis=1))
    assert bad.size == 0, f"first differing node: gpu {gn[bad[0]]} oracle {on[bad[0]]}"
    assert np.array_equal(gs, os_)


def assert_same_run(g, o):
    assert g["n_iter"] == o["n_iter"]
    assert np.array_equal(g["decision"], o["decision"])
    assert np.array_equal(g["hits"], o["hits"])
    k = g["n_iter"]
    gh, oh = g["imp_history"][:k], o["imp_history"][:k]
    assert np.array_equal(np.isnan(gh), np.isnan(oh))
    assert np.array_equal(gh[~np.isnan(gh)], oh[~np.isnan(oh)])
    assert np.array_equal(g["shadow_max"][:k], o["shadow_max"][:k])
    if "rank" in g and "rank" in o:
        assert np.array_equal(g["rank"], o["rank"])
    if g.get("traces") and o.get("traces"):
        assert len(g["traces"]) == len(o["traces"])
        for gt, ot in zip(g["traces"], o["traces"]):
            assert_same_trace(gt, ot)
