"""Pins for the CPU oracle: checks against facts fixed by the paper's definitions
and by mathematics, not against the oracle's own formulas.

* brute force on tiny inputs through a different route (pairwise join of two
  length-m sequences, scipy z-scores, explicit vector differences, Python loops)
* the l = m special case, which reduces to the z-normalised Euclidean distance
  profile (numpy's Pearson correlation)
* invariants: MPdist(A,A)=0, symmetry, range [0, 2 sqrt(l)], D_s(s*m)=0,
  invariance under T -> aT+b
* planted exact repeats, recovered by the greedy search with zero area
* hand-worked greedy / neighbours / criterion examples
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2401_13680_amd import synth


# ----------------------------------------------------------------- brute force
def _z(v):
    s = np.std(v)
    return np.zeros_like(v) if s <= 1e-6 * max(1.0, np.max(np.abs(v))) else stats.zscore(v)


def brute_mpdist(A, B, l, k):
    """MPdist of two equal-length sequences as a join: for every l-subsequence
    of A its nearest neighbour distance in B (P_AB), and vice versa (P_BA);
    the k-th smallest of the union (largest if there are no more than k)."""
    m = len(A)
    w = m - l + 1
    za = [_z(A[i:i + l]) for i in range(w)]
    zb = [_z(B[i:i + l]) for i in range(w)]
    P_AB = [min(float(np.linalg.norm(za[i] - zb[j])) for j in range(w)) for i in range(w)]
    P_BA = [min(float(np.linalg.norm(zb[j] - za[i])) for i in range(w)) for j in range(w)]
    allv = sorted(P_AB + P_BA)
    return allv[k - 1] if len(allv) > k else allv[-1]


def brute_profile_set(x, m, l, k, series_stats=True):
    n = len(x)
    out = []
    for s in range(n // m):
        A = x[s * m: s * m + m]
        out.append([brute_mpdist(A, x[j:j + m], l, k) for j in range(n - m + 1)])
    return np.array(out)


@pytest.mark.parametrize("n,m,l,k,seed", [
    (60, 12, 6, 2, 0), (64, 16, 5, 3, 1), (50, 10, 10, 1, 2), (70, 14, 2, 4, 3),
    (45, 9, 4, 20, 4), (66, 11, 7, 1, 5), (80, 20, 13, 5, 6),
])
def test_profile_set_matches_bruteforce_join(n, m, l, k, seed):
    x = synth.random_tiny(n, seed)
    D = oracle.profile_set(x, m, l, k)
    B = brute_profile_set(x, m, l, k)
    assert D.shape == B.shape == (n // m, n - m + 1)
    # compare squared distances: sqrt amplifies rounding near zero
    np.testing.assert_allclose(D ** 2, B ** 2, rtol=0, atol=1e-9)


def test_bruteforce_catches_dropped_column_minima():
    """A plausible mistake (profile from allP_AB only) fails the brute-force pin."""
    x = synth.random_tiny(60, 11)
    m, l, k = 12, 6, 2
    Z = oracle.znorm_matrix(x, l)
    w = m - l + 1
    E = oracle.ed_matr(Z[:w], Z)
    ab = np.lib.stride_tricks.sliding_window_view(E, w, axis=1).min(axis=2)
    wrong = np.sort(ab.T, axis=1)[:, k - 1]
    B = brute_profile_set(x, m, l, k)[0]
    assert np.max(np.abs(wrong - B)) > 1e-3


# --------------------------------------------------------- l = m closed form
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_l_equals_m_is_znormalised_distance_profile(seed):
    x = synth.random_tiny(300, seed)
    m = 25
    D = oracle.profile_set(x, m, m, 3)
    for s in range(len(x) // m):
        q = x[s * m:(s + 1) * m]
        r = np.array([np.corrcoef(q, x[j:j + m])[0, 1] for j in range(len(x) - m + 1)])
        ref = np.sqrt(np.maximum(2.0 * m * (1.0 - r), 0.0))
        np.testing.assert_allclose(D[s], ref, atol=2e-6)


# ------------------------------------------------------------------ invariants
def test_invariants():
    x = synth.regime_series(3000, 7, len_range=(400, 900)).x
    m, l = 60, 30
    k = oracle.default_k(m)
    D = oracle.profile_set(x, m, l, k)
    nseg = len(x) // m
    assert D.shape == (nseg, len(x) - m + 1)
    assert np.all(D >= 0) and np.all(D <= 2 * math.sqrt(l) + 1e-9)
    for s in range(nseg):
        assert D[s, s * m] < 1e-6                 # a segment is its own window
    # affine invariance
    D2 = oracle.profile_set(3.5 * x - 17.0, m, l, k)
    np.testing.assert_allclose(D2, D, atol=1e-6)
    # symmetry MPdist(A,B) == MPdist(B,A)
    rng = np.random.default_rng(3)
    for _ in range(20):
        i, j = rng.integers(0, len(x) - m, size=2)
        a, b = x[i:i + m], x[j:j + m]
        assert abs(oracle.mpdist(a, b, l, k) - oracle.mpdist(b, a, l, k)) < 1e-9
        assert oracle.mpdist(a, a, l, k) < 1e-6


def test_k_at_least_2w_takes_the_largest():
    x = synth.random_tiny(40, 9)
    m, l = 10, 8                     # w = 3, 2w = 6
    big = oracle.profile_set(x, m, l, 6)
    bigger = oracle.profile_set(x, m, l, 50)
    np.testing.assert_array_equal(big, bigger)
    B = brute_profile_set(x, m, l, 6)
    np.testing.assert_allclose(big ** 2, B ** 2, atol=1e-9)


def test_constant_windows():
    """A constant subsequence is the zero vector after z-normalisation:
    const vs const is distance 0, const vs non-constant is sqrt(l)."""
    rng = np.random.default_rng(0)
    x = np.concatenate([np.full(20, 2.0), rng.normal(size=20), np.full(20, -1.0)])
    l = 5
    Z = oracle.znorm_matrix(x, l)
    E = oracle.ed_matr(Z[:3], Z)
    assert np.allclose(E[0, 40:56], 0.0)
    assert np.allclose(E[0, 22:30], math.sqrt(l))


# -------------------------------------------------------------- planted repeats
def test_planted_repeats_recovered():
    m, l = 40, 20
    x, order = synth.planted_motifs(m, 3, [3, 2, 4], seed=1)
    k = oracle.default_k(m)
    r = oracle.snippets(x, m, l, K=3, k=k)
    first_copy = {int(np.flatnonzero(order == mid)[0]) for mid in range(3)}
    assert set(r["picks"]) == first_copy
    a = r["areas"]
    assert a[0] > a[1] > a[2] > 0        # windows straddling two motifs stay > 0
    D = r["D"]
    M = D[r["picks"]].min(axis=0)
    assert np.all(M[::m][:len(order)] < 1e-6)   # every segment-aligned window is matched
    for s in range(len(order)):
        for t in range(len(order)):
            if order[s] == order[t]:
                assert D[s, t * m] < 1e-6      # copies score zero against each other
    # a 4th pick can only be a second copy: it does not lower the area
    r4 = oracle.snippets(x, m, l, K=4, k=k)
    assert abs(r4["areas"][3] - r4["areas"][2]) < 1e-6


# ---------------------------------------------------- hand-worked selection
def test_greedy_neighbours_hand_example():
    D = np.array([[0.0, 4.0, 4.0],
                  [4.0, 0.0, 4.0],
                  [1.0, 1.0, 1.0]])
    picks, areas = oracle.greedy(D, 2)
    # step 1: areas 8, 8, 3 -> segment 2; step 2: 2 vs 2, tie -> segment 0
    assert picks == [2, 0] and areas == [3.0, 2.0]
    owner, frac = oracle.neighbours(D, picks)
    assert list(owner) == [1, 0, 0]
    assert np.allclose(frac, [2 / 3, 1 / 3])
    # with equal values the earliest pick owns the window
    owner2, _ = oracle.neighbours(np.array([[1.0, 2.0], [1.0, 1.0]]), [1, 0])
    assert list(owner2) == [0, 0]


def test_snippet_order_by_frac():
    D = np.array([[0.0, 9.0, 9.0, 9.0],
                  [5.0, 0.0, 0.0, 0.0],
                  [9.0, 9.0, 9.0, 0.5]])
    r = oracle.snippets(None, 1, 1, K=2, D=D)
    # greedy: areas 27, 5, 27.5 -> 1 first, then 0 (area 0 < 4.5)
    assert r["picks"] == [1, 0]
    assert [rec["segment"] for rec in r["records"]] == [1, 0]
    assert [rec["frac"] for rec in r["records"]] == [0.75, 0.25]


def test_criterion_hand_example():
    D = np.array([[0.0, 1.0, 2.0],
                  [2.0, 2.0, 0.0],
                  [4.0, 0.0, 0.0]])
    # pairs (0,1) and (1,0): |0-2|+|1-2|+|2-0| = 5 each -> 10; max D = 4
    assert oracle.criterion(D, [0, 1]) == pytest.approx(2.5)
    assert oracle.criterion(D, [1]) == 0.0
    # three snippets: (0,1)=5, (0,2)=4+1+2=7, (1,2)=2+2+0=4 -> 2*16/4
    assert oracle.criterion(D, [0, 1, 2]) == pytest.approx(8.0)


def test_select_length_prefers_distinct_shapes():
    """Series of two alternating motif shapes of length 50: at m=50 the two
    snippets are distinct shapes, so their profiles differ most."""
    m0 = 50
    x, _ = synth.planted_motifs(m0, 2, [4, 4], seed=5, noise=0.01)
    res = oracle.select_length(x, [25, 50], K=2)
    assert res["m_best"] == 50
    assert all(s >= 0 for s in res["scores"])


def test_default_k_matches_five_percent_of_2m():
    for m in range(2, 5001):
        assert oracle.default_k(m) == math.ceil(round(0.05 * 2 * m, 9))


def test_local_pairs_equal_full_profile():
    x = synth.regime_series(3000, 17, len_range=(300, 900)).x
    m, l, k = 60, 30, 6
    D = oracle.profile_set(x, m, l, k)
    rng = np.random.default_rng(1)
    pairs = [(int(rng.integers(D.shape[0])), int(rng.integers(D.shape[1]))) for _ in range(30)]
    got = oracle.mpdist_pairs_local(x, m, l, k, pairs)
    np.testing.assert_allclose(got ** 2, [D[s, j] ** 2 for s, j in pairs], atol=1e-9)


def test_samples_equal_full_profile():
    """mpdist_samples (each entry from its own w x w block of ED_matr, the
    checker of the full-size GPU test) equals the whole profile set entry for
    entry, including the first and last segment and window."""
    x = synth.regime_series(3000, 18, len_range=(300, 900)).x
    m, l, k = 60, 30, 6
    D = oracle.profile_set(x, m, l, k)
    rng = np.random.default_rng(2)
    nseg, Nm = D.shape
    pairs = [(int(rng.integers(nseg)), int(rng.integers(Nm))) for _ in range(40)]
    pairs += [(0, 0), (nseg - 1, Nm - 1), (nseg - 1, 0), (0, Nm - 1), (7, 7 * m)]
    got = oracle.mpdist_samples(x, m, l, k, pairs)
    np.testing.assert_array_equal(got, [D[s, j] for s, j in pairs])
