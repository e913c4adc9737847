"""Degenerate sizes of the method against the FP64 oracle: one segment and one
window (n = m), one segment with a ragged tail (n = 2m - 1), the smallest m
and l (w = 1), every segment chosen (K = n/m), an empty series and sizes the
library must refuse.  Profiles to the stated tolerance, snippets exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _check(x, m, l, K):
    print(f"edge: n={len(x)} m={m} l={l} K={K}", flush=True)
    g = api.snippets(dev(x), m, l, K, profiles=True, owner=True)
    r = oracle.snippets(x, m, l, K)
    assert [a["segment"] for a in g["records"]] == [a["segment"] for a in r["records"]]
    assert [a["greedy_rank"] for a in g["records"]] == [a["greedy_rank"] for a in r["records"]]
    P = g["profiles"].cpu().numpy().astype(np.float64)
    Pr = r["D"][list(r["picks"])]
    e = np.abs(P * P - Pr * Pr) / (4.0 * l)
    assert e.max() <= 1e-4
    D, _ = api.profile_set(dev(x), m, l)
    assert D.shape == r["D"].shape
    e = np.abs(D.cpu().numpy().astype(np.float64) ** 2 - r["D"] ** 2) / (4.0 * l)
    assert e.max() <= 1e-4
    return g, r


def test_one_segment_one_window():
    x = synth.random_tiny(64, 31)
    g, r = _check(x, 64, 32, 1)
    assert g["records"][0]["segment"] == 0 and g["records"][0]["frac"] == 1.0
    assert g["profiles"].shape == (1, 1) and float(g["profiles"][0, 0]) <= 1e-2   # the segment against itself


def test_one_segment_ragged_tail():
    x = synth.random_tiny(2 * 50 - 1, 32)
    g, r = _check(x, 50, 25, 1)
    assert g["owner"].numel() == 50


def test_smallest_window_w_equals_one():
    # m = l = 2: every distance is 0 or 2 sqrt(2) in exact arithmetic, so the
    # greedy search meets exact ties that FP32 rounding of rho near 1 breaks
    # (sqrt turns it into distances of about 1e-3); only the profiles are
    # compared there.  With l = 20 the snippets are compared as well.
    x = synth.random_tiny(400, 33)
    D, _ = api.profile_set(dev(x), 2, 2)
    ref = oracle.profile_set(x, 2, 2)
    e = np.abs(D.cpu().numpy().astype(np.float64) ** 2 - ref ** 2) / 8.0
    assert D.shape == ref.shape and e.max() <= 1e-4
    _check(synth.random_tiny(600, 34), 20, 20, 4)


def test_every_segment_chosen():
    x = synth.regime_series(1200, 35, len_range=(200, 400)).x
    g, r = _check(x, 60, 30, 20)          # K = n/m = 20
    assert sorted(a["segment"] for a in g["records"]) == list(range(20))
    assert abs(sum(a["frac"] for a in g["records"]) - 1.0) < 1e-12


def test_refused_sizes():
    x = dev(synth.random_tiny(500, 36))
    for m, l, K in ((1, 1, 1), (600, 300, 1), (50, 1, 1), (50, 51, 1), (50, 25, 0), (50, 25, 11)):
        with pytest.raises(PstError):
            api.snippets(x, m, l, K)
    with pytest.raises(PstError):
        api.profile_set(dev(np.zeros(0)), 10, 5)
