"""The margin-aware greedy comparison itself, on the oracle's own profiles
(CPU): identical profiles always agree; a perturbation inside the bound may
flip a near-tie; a planted wrong pick outside the bound is caught."""
import numpy as np
import pytest

import oracle
from greedy_bounds import areas_from_profiles, check_greedy
from paper_2401_13680_amd import synth


def _setup():
    x = synth.four_regimes(1).x
    D = oracle.profile_set(x, 100, 50, 10)
    rows = {s: D[s] for s in range(D.shape[0])}
    return D, rows


def test_identical_profiles_give_the_oracle_picks():
    D, rows = _setup()
    picks, areas = oracle.greedy(D, 3)
    res = check_greedy(picks, rows, rows, list(rows), "same")
    assert all(eq for _, _, eq in res)
    assert all(B == 0.0 for _, B, _ in res)
    np.testing.assert_allclose(areas_from_profiles(D[picks]), areas, rtol=1e-12)


def test_perturbation_within_bound_is_accepted():
    D, rows = _setup()
    rng = np.random.default_rng(3)
    Dg = D + rng.uniform(-1e-3, 1e-3, size=D.shape)
    picks_g, _ = oracle.greedy(Dg, 3)
    res = check_greedy(picks_g, {s: Dg[s] for s in rows}, rows, list(rows), "noisy")
    assert len(res) == 3


def test_wrong_pick_outside_bound_is_caught():
    D, rows = _setup()
    picks, _ = oracle.greedy(D, 3)
    wrong = [picks[0], picks[2], picks[1]]          # second and third swapped
    with pytest.raises(AssertionError):
        check_greedy(wrong, rows, rows, list(rows), "planted")
