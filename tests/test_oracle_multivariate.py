"""Pins of the oracle's multivariate reading: section 3.2 searches every
coordinate of a d-coordinate series (eqs. 1-2) on its own.  The pins follow
from that statement and from the z-normalisation of the distance, not from
the oracle's own code: identical coordinates give identical results, a
positively rescaled and shifted coordinate gives the same snippets, a change
to one coordinate leaves the others alone, and reordering the coordinates
reorders the results.  A planted mistake (every coordinate searched on
coordinate 0) fails them."""
import numpy as np

import oracle
from paper_2401_13680_amd import synth

M, L, K = 60, 30, 3


def _segments(r):
    return [(a["segment"], a["greedy_rank"], a["frac"]) for a in r["records"]]


def _series(d, seed):
    return synth.multivariate_series(1800, d, seed, len_range=(300, 700)).x


def _check_pins(multi):
    X = _series(3, 12)
    R = multi(X, M, L, K)
    assert len(R) == 3
    # each coordinate's result is the univariate search of that coordinate
    for j in range(3):
        assert _segments(R[j]) == _segments(oracle.snippets(X[j], M, L, K))
    # reordering the coordinates reorders the results
    Rr = multi(X[::-1].copy(), M, L, K)
    for j in range(3):
        assert _segments(Rr[j]) == _segments(R[2 - j])
    # replacing coordinate 1 leaves coordinates 0 and 2 alone
    X2 = X.copy()
    X2[1] = np.random.default_rng(0).normal(size=X.shape[1])
    R2 = multi(X2, M, L, K)
    for j in (0, 2):
        assert _segments(R2[j]) == _segments(R[j])
        assert np.array_equal(R2[j]["D"], R[j]["D"])


def test_coordinates_searched_independently():
    _check_pins(oracle.snippets_multi)


def test_identical_coordinates_identical_results():
    x = _series(1, 3)[0]
    R = oracle.snippets_multi(np.stack([x, x, x]), M, L, K)
    for r in R[1:]:
        assert _segments(r) == _segments(R[0])
        assert np.array_equal(r["D"], R[0]["D"])
        assert np.array_equal(r["owner"], R[0]["owner"])


def test_affine_copy_same_snippets():
    # z-normalised distances do not change under x -> a x + b with a > 0
    x = _series(1, 5)[0]
    R = oracle.snippets_multi(np.stack([x, 3.5 * x - 40.0]), M, L, K)
    assert _segments(R[1]) == _segments(R[0])
    np.testing.assert_allclose(R[1]["D"] ** 2, R[0]["D"] ** 2, rtol=0, atol=1e-9)


def test_planted_mistake_fails_the_pins():
    def wrong(X, m, l, K, k=None):
        return [oracle.snippets(X[0], m, l, K, k) for _ in range(X.shape[0])]

    try:
        _check_pins(wrong)
    except AssertionError:
        return
    raise AssertionError("a multivariate search that ignores the coordinates passed the pins")
