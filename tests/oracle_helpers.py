"""Test-side reconstruction helpers (pure Python/numpy) used to pin the
oracle's importance arithmetic.  They rebuild the widened matrix of one
iteration from the oracle's own binning and keyed permutations, which are
pinned separately, and route rows through traced trees."""
from fractions import Fraction

import numpy as np

from oracle import oracle as O


def widened(X, state, t, seed, n_bins):
    bins, _, _ = O.bin_matrix(X, n_bins)
    n = X.shape[0]
    active = [j for j in range(X.shape[1]) if state[j] >= 0]
    n_sha = len(active)
    while n_sha < 5:
        n_sha *= 2
    cols = [bins[j] for j in active]
    for s in range(n_sha):
        src = bins[active[s % len(active)]]
        perm = [O.keyed_perm(seed, O.STREAM_SHADOW, t, s, 0, 0, n, i) for i in range(n)]
        cols.append(src[perm])
    return np.stack(cols), active, n_sha


def tree_dict(nodes, tree):
    return {int(r[1]): r for r in nodes if int(r[0]) == tree}


def leaf_of(td, W, row, sub_f=-1, sub_b=0):
    h = 1
    while int(td[h][2]) >= 0:
        f = int(td[h][2])
        b = sub_b if f == sub_f else int(W[f][row])
        h = 2 * h if b <= int(td[h][3]) else 2 * h + 1
    return h


def route_counts(td, W, rows, w, y, K):
    """Weighted class counts reaching every node of a traced tree."""
    cnt = {h: np.zeros(K, dtype=np.int64) for h in td}
    for i in rows:
        h = 1
        while True:
            cnt[h][y[i]] += int(w[i])
            if int(td[h][2]) < 0:
                break
            h = 2 * h if int(W[int(td[h][2])][i]) <= int(td[h][3]) else 2 * h + 1
    return cnt


def gini_decrease_fraction(cp, cl, cr):
    def s_over_n(c):
        return Fraction(int((c * c).sum()), int(c.sum()))
    return s_over_n(cl) + s_over_n(cr) - s_over_n(cp)
