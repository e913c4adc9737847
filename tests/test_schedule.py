"""Scheduling of section 4.2 (host only, no GPU): the oracle's run-time
regression and Karmarkar-Karp partition against what the mathematics fixes,
then the library's pst_model_* / pst_partition_* against the oracle."""
import itertools

import numpy as np
import pytest

from oracle import schedule as SC
from paper_2401_13680_amd import api
from paper_2401_13680_amd._lib import PstError

# ---------------------------------------------------------------- oracle pins


def test_kk_two_way_textbook_example():
    # differencing 8,7,6,5,4: 8-7=1; 6-5=1; 4-1=3; 3-1=2; 2-1... final difference 2
    part, load = SC.kk_partition([8, 7, 6, 5, 4], 2)
    assert load == [16.0, 14.0]
    assert sum(c for c, p in zip([8, 7, 6, 5, 4], part) if p == 0) == 16


def test_kk_two_way_difference_at_most_largest_item():
    # each differencing step leaves a number no larger than the current
    # largest, so the final difference never exceeds the largest cost
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.integers(1, 100, size=int(rng.integers(2, 12))).tolist()
        part, load = SC.kk_partition(c, 2)
        assert load[0] - load[1] <= max(c)
        assert load[0] >= load[1]


def test_kk_invariants_and_special_cases():
    rng = np.random.default_rng(2)
    for _ in range(40):
        k = int(rng.integers(1, 6))
        c = rng.uniform(0, 10, size=int(rng.integers(0, 15))).tolist()
        part, load = SC.kk_partition(c, k)
        assert len(load) == k and all(0 <= p < k for p in part)
        for j in range(k):
            assert abs(load[j] - sum(x for x, p in zip(c, part) if p == j)) < 1e-9
        assert load == sorted(load, reverse=True)
    # no more items than parts: one item per part
    part, load = SC.kk_partition([5.0, 3.0, 9.0], 4)
    assert sorted(part) == sorted(set(part)) and sorted(load) == [0.0, 3.0, 5.0, 9.0]
    # equal items, a multiple of the parts: perfectly balanced
    part, load = SC.kk_partition([2.0] * 12, 4)
    assert load == [6.0] * 4
    # one part: everything in it
    assert SC.kk_partition([1.0, 2.0], 1) == ([0, 0], [3.0])


def test_kk_brute_force_small():
    # a heuristic: never better than the optimum, and optimal on these sets
    for c in ([3, 1, 1, 2, 2, 1], [7, 5, 4, 3, 1], [10, 10, 9, 1, 1]):
        best = min(max(sum(x for x, s in zip(c, a) if s == 0), sum(x for x, s in zip(c, a) if s == 1))
                   for a in itertools.product([0, 1], repeat=len(c)))
        assert SC.kk_partition(c, 2)[1][0] >= best
    assert SC.kk_partition([3, 1, 1, 2, 2, 1], 2)[1] == [5.0, 5.0]


def test_kk_planted_mistake_fails_textbook():
    # merging largest with largest instead of largest with smallest
    def wrong(costs, k):
        t = sorted(([float(c)] + [0.0] * (k - 1) for c in costs), key=lambda s: -(s[0] - s[-1]))
        while len(t) > 1:
            a, b = t.pop(0), t.pop(0)
            s = sorted((a[j] + b[j] for j in range(k)), reverse=True)
            t.append(s)
            t.sort(key=lambda s: -(s[0] - s[-1]))
        return t[0]
    assert wrong([8, 7, 6, 5, 4], 2) != [16.0, 14.0]


def _poly_runs(D, coef, configs):
    return [(n, m, l, float(SC.design_row(D, n, m, l) @ coef)) for n, m, l in configs]


def _configs(rng, count):
    out = []
    while len(out) < count:
        n = int(rng.integers(20_000, 400_000))
        m = int(rng.integers(32, 600))
        l = int(rng.integers(2, m + 1))
        out.append((n, m, l))
    return out


def test_regression_recovers_an_exact_polynomial():
    rng = np.random.default_rng(3)
    for D in (1, 2, 3):
        P = len(SC.monomial_exponents(D))
        assert P == (D + 1) * (D + 2) * (D + 3) // 6
        coef = rng.uniform(0.5, 2.0, size=P)
        runs = _poly_runs(D, coef, _configs(rng, 3 * P))
        got = SC.fit(D, runs)
        for n, m, l in _configs(rng, 10):
            want = float(SC.design_row(D, n, m, l) @ coef)
            assert abs(SC.predict(D, got, n, m, l) - want) <= 1e-5 * want


def test_regression_planted_mistake_fails():
    # a fit without the constant monomial cannot reproduce a cubic that has one
    rng = np.random.default_rng(4)
    D = 2
    coef = rng.uniform(0.5, 2.0, size=len(SC.monomial_exponents(D)))
    runs = _poly_runs(D, coef, _configs(rng, 30))
    A = np.array([SC.design_row(D, n, m, l)[1:] / ms for n, m, l, ms in runs])
    c, *_ = np.linalg.lstsq(A, np.ones(len(runs)), rcond=None)
    n, m, l = 123_456, 200, 100
    want = float(SC.design_row(D, n, m, l) @ coef)
    assert abs(float(SC.design_row(D, n, m, l)[1:] @ c) - want) > 1e-3 * want


# ---------------------------------------------------------------- library vs oracle


def test_library_kk_equals_oracle():
    rng = np.random.default_rng(5)
    for trial in range(60):
        k = int(rng.integers(1, 9))
        cnt = int(rng.integers(0, 40))
        c = (rng.integers(0, 20, size=cnt).astype(float) if trial % 2 else rng.uniform(0, 50, size=cnt)).tolist()
        assert api.partition_kk(c, k) == SC.kk_partition(c, k), (k, c)


def test_library_model_equals_oracle():
    rng = np.random.default_rng(6)
    for D in (1, 2, 3):
        runs = [(n, m, l, float(rng.uniform(1.0, 200.0))) for n, m, l in _configs(rng, 25)]
        M = api.RuntimeModel(D)
        for r in runs:
            M.observe(*r)
        M.fit()
        ref = SC.fit(D, runs)
        assert len(M.coefficients()) == len(ref)
        for n, m, l in [r[:3] for r in runs] + _configs(rng, 10):
            want = SC.predict(D, ref, n, m, l)
            assert abs(M.predict(n, m, l) - want) <= 1e-6 * max(1.0, abs(want))


def test_library_partition_lengths_uses_predictions():
    rng = np.random.default_rng(7)
    M = api.RuntimeModel(2)
    runs = [(n, m, m // 2, 1e-6 * (n // m) * (m - m // 2 + 1) * (n - m // 2 + 1)) for n, m, _ in _configs(rng, 20)]
    for r in runs:
        M.observe(*r)
    M.fit()
    ms = list(range(64, 513, 32))
    pred = [max(M.predict(250_000, m, m // 2), 0.0) for m in ms]
    assert api.partition_lengths(M, 250_000, ms, 4) == SC.kk_partition(pred, 4)


def test_library_errors():
    with pytest.raises(PstError):
        api.RuntimeModel(0)
    with pytest.raises(PstError):
        api.RuntimeModel(5)
    M = api.RuntimeModel(1)
    with pytest.raises(PstError):
        M.fit()                      # nothing observed
    with pytest.raises(PstError):
        M.predict(1000, 100, 50)     # not fitted
    with pytest.raises(PstError):
        M.observe(1000, 100, 50, -1.0)
    with pytest.raises(PstError):
        M.observe(1000, 100, 200, 1.0)
    with pytest.raises(PstError):
        api.partition_kk([1.0, -2.0], 2)
    with pytest.raises(PstError):
        api.partition_kk([1.0, float("nan")], 2)
    with pytest.raises(PstError):
        api.partition_kk([1.0], 0)
    with pytest.raises(PstError):
        api.partition_kk([1.0] * 5000, 4096)   # 5000 x 4096 slots > 2^24
