"""GPU parity of the multivariate search (every coordinate of eqs. 1-2
searched on its own, section 3.2; one batched profile launch for all
coordinates).  Against the FP64 oracle: snippet indices, greedy order and
neighbour counts exactly, with the window owners compared wherever the two
nearest snippets' profiles differ by more than the FP32 profile tolerance.
Against one pst_snippets call per coordinate: bit-identical records, owners
and maxima."""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError, Snippet

pytestmark = pytest.mark.gpu


def _assert_same_as_single(X, R, m, l, K):
    for j in range(X.shape[0]):
        s = api.snippets(X[j], m, l, K, owner=True)
        assert R[j]["records"] == s["records"], j
        assert torch.equal(R[j]["owner"], s["owner"]), j
        assert R[j]["dmax"] == s["dmax"], j


def test_multi_matches_oracle_and_single_calls():
    S = synth.multivariate_series(6000, 3, 11, len_range=(800, 2000))
    m, l, K = 100, 50, 3
    print("multi: n=6000 d=3 m=100 l=50 K=3", flush=True)
    X = torch.from_numpy(S.x).cuda()
    R = api.snippets_multi(X, m, l, K, owner=True)
    ref = oracle.snippets_multi(S.x, m, l, K)
    for j in range(3):
        g, r = R[j], ref[j]
        assert [a["segment"] for a in g["records"]] == [a["segment"] for a in r["records"]], j
        assert [a["greedy_rank"] for a in g["records"]] == [a["greedy_rank"] for a in r["records"]], j
        # owners where the nearest snippet is clear of the second by the
        # profile tolerance (1e-4 of the distance range 2 sqrt(l))
        P = np.sort(r["D"][list(r["picks"])], axis=0)
        clear = (P[1] - P[0]) > 2e-4 * math.sqrt(l) if len(P) > 1 else np.ones(P.shape[1], bool)
        own = g["owner"].cpu().numpy()
        assert np.array_equal(own[clear], r["owner"][clear]), j
        if clear.all():
            assert [a["frac"] for a in g["records"]] == [a["frac"] for a in r["records"]], j
        assert abs(g["dmax"] - float(r["D"].max())) <= 1e-4 * float(r["D"].max())
    _assert_same_as_single(X, R, m, l, K)


def test_multi_ragged_sizes_equal_single_calls():
    # five coordinates, n not a multiple of m, tiles with a ragged tail
    S = synth.multivariate_series(30_011, 5, 13)
    m, l, K = 128, 64, 4
    print("multi: n=30011 d=5 m=128 l=64 K=4", flush=True)
    X = torch.from_numpy(S.x).cuda()
    R = api.snippets_multi(X, m, l, K, owner=True)
    _assert_same_as_single(X, R, m, l, K)
    # a strided view (ld > n) gives the same result
    W = torch.zeros((5, 30_100), dtype=torch.float64, device="cuda")
    W[:, :30_011] = X
    R2 = api.snippets_multi(W[:, :30_011], m, l, K, owner=True)
    for a, b in zip(R, R2):
        assert a["records"] == b["records"] and torch.equal(a["owner"], b["owner"])


def test_multi_errors():
    S = synth.multivariate_series(3000, 3, 14, len_range=(500, 900))
    X = torch.from_numpy(S.x).cuda()
    ctx = api.context(0)
    L = ctx.L
    assert L.pst_snippets_multi_workspace_bytes(0, 3000, 100, 50, 3) == 0
    assert L.pst_snippets_multi_workspace_bytes(17, 3000, 100, 50, 3) == 0
    nb = L.pst_snippets_multi_workspace_bytes(3, 3000, 100, 50, 3)
    assert nb > 0
    ws = ctx.workspace(nb)
    recs = (Snippet * 9)()
    p = ctypes.c_void_p
    # ld < n
    rc = L.pst_snippets_multi(ctx.h, p(X.data_ptr()), 3, 2999, 3000, 100, 50, 0, 3, recs, None, None,
                              p(ws.data_ptr()), ws.numel())
    assert rc != 0
    # workspace too small
    rc = L.pst_snippets_multi(ctx.h, p(X.data_ptr()), 3, 3000, 3000, 100, 50, 0, 3, recs, None, None,
                              p(ws.data_ptr()), nb - 256)
    assert rc != 0
    # a non-finite value in coordinate 2 is reported by coordinate
    Y = X.clone()
    Y[2, 1234] = float("nan")
    with pytest.raises(PstError, match="coordinate 2"):
        api.snippets_multi(Y, 100, 50, 3)
    # the context still works
    R = api.snippets_multi(X, 100, 50, 3)
    assert len(R) == 3
