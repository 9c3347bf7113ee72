"""Pins of the oracle's random streams (test infrastructure).

Philox4x32-10 is pinned against published known-answer vectors and against
rocRAND's independent open-source engine; the keyed bijection and the
bootstrap against the properties that define them (bijectivity, uniformity,
multinomial draw counts)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in _kat_rows():
        assert [int(x) for x in O.philox(ctr, key)] == want


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.check_call(["hipcc", "-O1", os.path.join(HERE, "kat", "rocrand_philox_kat.cpp"),
                           "-o", exe])
    return exe


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(5)
    cases = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    cases[:, 1] &= (1 << 30) - 1  # the engine reaches counter word 1 through 4*offset
    text = "\n".join(" ".join(f"{int(v):08x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_kat], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        want = [int(x, 16) for x in line.split()]
        assert [int(x) for x in O.philox(c[:4], c[4:6])] == want


@pytest.mark.parametrize("m", list(range(1, 70)) + [255, 256, 257, 1000, 1023, 1025, 4097])
def test_keyed_perm_is_bijection(m):
    for stream, seed, a in [(3, 1, 0), (2, 7001, 5), (4, 2**40 + 3, 17)]:
        img = [O.keyed_perm(seed, stream, 3, a, 9, 0, m, x) for x in range(m)]
        assert sorted(img) == list(range(m))


def test_keyed_perm_bijection_large():
    m = 40000
    img = np.array([O.keyed_perm(99, 3, 1, 2, 0, 0, m, x) for x in range(m)])
    assert np.array_equal(np.sort(img), np.arange(m))


def test_keyed_perm_uniform_image():
    # pi(0) over independent keys must be uniform on [0, m)
    m, reps = 10, 4000
    img = [O.keyed_perm(1234, 2, 1, tree, 1, 0, m, 0) for tree in range(reps)]
    counts = np.bincount(img, minlength=m)
    assert stats.chisquare(counts).pvalue > 1e-4


@pytest.mark.parametrize("m", [2, 3, 5, 10, 37, 200])
def test_keyed_perm_uniform_pairs(m):
    # (pi(x0), pi(x1)) over independent keys: uniform over the m(m-1) ordered
    # pairs.  Narrow Feistel halves are where a too-short network shows bias.
    reps = 250 * m * (m - 1) if m <= 10 else 20000
    x0, x1 = 0, m - 1
    a = np.array([O.keyed_perm(77, 4, 2, tr, 3, 0, m, x0) for tr in range(reps)])
    b = np.array([O.keyed_perm(77, 4, 2, tr, 3, 0, m, x1) for tr in range(reps)])
    assert np.all(a != b)
    if m > 37:  # too many cells for a pair table: test each margin and the sum
        assert stats.chisquare(np.bincount(a, minlength=m)).pvalue > 1e-4
        assert stats.chisquare(np.bincount((a + b) % m, minlength=m)).pvalue > 1e-4
        return
    counts = np.bincount(a * m + b, minlength=m * m).reshape(m, m)
    off = counts[~np.eye(m, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-4


def test_keyed_perm_streams_differ():
    m = 1000
    a = [O.keyed_perm(5, 3, 1, 0, 0, 0, m, x) for x in range(50)]
    b = [O.keyed_perm(5, 3, 2, 0, 0, 0, m, x) for x in range(50)]
    c = [O.keyed_perm(5, 2, 1, 0, 0, 0, m, x) for x in range(50)]
    assert a != b and a != c


def test_bootstrap_is_multinomial():
    n = 5000
    w = O.bootstrap(7, 1, 0, n)
    assert w.sum() == n
    # fraction out of bag -> (1 - 1/n)^n ~ e^-1
    oob = np.mean(w == 0)
    assert abs(oob - (1 - 1 / n) ** n) < 0.02
    # multiplicity histogram against Binomial(n, 1/n)
    counts = np.bincount(w, minlength=6)[:5].astype(float)
    probs = stats.binom.pmf(np.arange(5), n, 1 / n)
    exp = probs * n
    chi = ((counts - exp) ** 2 / exp).sum()
    assert chi < stats.chi2.ppf(0.9999, 4)
    # draws are uniform over rows: pooled over trees, row totals ~ Poisson
    tot = sum(O.bootstrap(7, 1, tree, 200).astype(np.int64) for tree in range(400))
    assert stats.chisquare(tot).pvalue > 1e-4


def test_bootstrap_keyed():
    a = O.bootstrap(7, 1, 0, 300)
    assert np.array_equal(a, O.bootstrap(7, 1, 0, 300))
    assert not np.array_equal(a, O.bootstrap(7, 1, 1, 300))
    assert not np.array_equal(a, O.bootstrap(7, 2, 0, 300))
    assert not np.array_equal(a, O.bootstrap(8, 1, 0, 300))
