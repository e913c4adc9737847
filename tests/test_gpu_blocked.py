"""Bounded-memory snippet search (pst_snippets_blocked): the profile set is
recomputed every greedy round in blocks of segments and never held whole.
Every output must be bit-identical to pst_snippets', for any block size,
including one segment per block and a ragged last block; snippet indices
also match the FP64 oracle exactly."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError, Snippet

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a["records"] == b["records"]
    assert torch.equal(a["owner"], b["owner"])
    assert torch.equal(a["profiles"], b["profiles"])
    assert a["dmax"] == b["dmax"]


def test_blocked_equals_in_core_small():
    x = synth.four_regimes(1).x
    m, l, K = 100, 50, 3
    T = torch.from_numpy(x).cuda()
    ref = api.snippets(T, m, l, K, profiles=True, owner=True)
    gold = oracle.snippets(x, m, l, K)
    assert [r["segment"] for r in ref["records"]] == [r["segment"] for r in gold["records"]]
    for B in (1, 3, 7, 20):
        print(f"blocked: four_regimes seg_block={B}", flush=True)
        got = api.snippets_blocked(T, m, l, K, seg_block=B, profiles=True, owner=True)
        _same(got, ref)


def test_blocked_equals_in_core_bench_size():
    x = synth.workload_series("regimes5_n100000")
    m, l, K = 256, 128, 4
    T = torch.from_numpy(x).cuda()
    ref = api.snippets(T, m, l, K, profiles=True, owner=True)
    print("blocked: regimes5_n100000 seg_block=64 (390 = 6 x 64 + 6)", flush=True)
    got = api.snippets_blocked(T, m, l, K, seg_block=64, profiles=True, owner=True)
    _same(got, ref)
    # the budget form picks the largest block that fits
    budget = got["workspace_bytes"] + 1
    got2 = api.snippets_blocked(T, m, l, K, budget_bytes=budget, owner=True)
    assert got2["seg_block"] >= 64 and got2["workspace_bytes"] <= budget
    assert got2["records"] == ref["records"]


def test_blocked_sizes_and_errors():
    L = api.context(0).L
    n, m, l, K = 100_000, 256, 128, 4
    nseg = n // m
    assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, 0) == 0
    assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, nseg + 1) == 0
    sizes = [L.pst_snippets_blocked_workspace_bytes(n, m, l, K, b) for b in (1, 10, 100, nseg)]
    assert all(s > 0 for s in sizes) and sizes == sorted(sizes)
    assert L.pst_snippets_blocked_max_block(n, m, l, K, sizes[0] - 1) == 0
    b = L.pst_snippets_blocked_max_block(n, m, l, K, sizes[2])
    assert b >= 100
    assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, b) <= sizes[2]
    if b < nseg:
        assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, b + 1) > sizes[2]
    x = synth.four_regimes(1).x
    T = torch.from_numpy(x).cuda()
    with pytest.raises(PstError):
        api.snippets_blocked(T, 100, 50, 3, seg_block=21)
    bad = T.clone()
    bad[5] = float("nan")
    with pytest.raises(PstError):
        api.snippets_blocked(bad, 100, 50, 3, seg_block=4)
    r = api.snippets_blocked(T, 100, 50, 3, seg_block=4)
    assert len(r["records"]) == 3


def test_blocked_sweep_equals_in_core_sweep():
    x = synth.regime_series(20_000, 12, synth.SHAPES6, len_range=(1000, 3000)).x
    T = torch.from_numpy(x).cuda()
    ms, K = [40, 64, 96, 128], 3
    print("blocked sweep: n=20000 m in {40, 64, 96, 128} seg_block=37", flush=True)
    ref = api.select_length(T, ms, K, profiles=True, owner=True)
    got = api.select_length_blocked(T, ms, K, seg_block=37, profiles=True, owner=True)
    assert got["m_best"] == ref["m_best"]
    assert got["scores"] == ref["scores"]
    assert got["records"] == ref["records"]
    assert torch.equal(got["owner"], ref["owner"]) and torch.equal(got["profiles"], ref["profiles"])
    # the workspace is the largest candidate's, far below the batched sweep's
    L = api.context(0).L
    import ctypes
    arr = (ctypes.c_int32 * 4)(*ms)
    assert got["workspace_bytes"] < L.pst_select_length_workspace_bytes(20_000, arr, 4, None, K)


def test_spilled_equals_in_core():
    x = synth.workload_series("regimes5_n100000")
    m, l, K = 256, 128, 4
    T = torch.from_numpy(x).cuda()
    ref = api.snippets(T, m, l, K, profiles=True, owner=True)
    D, _ = api.profile_set(T, m, l)
    for B in (1, 64, 390):
        print(f"spilled: regimes5_n100000 seg_block={B}", flush=True)
        got = api.snippets_spilled(T, m, l, K, seg_block=B, profiles=True, owner=True)
        _same(got, ref)
        assert torch.equal(got["D_host"], D.cpu())   # the whole profile set, as computed in core
