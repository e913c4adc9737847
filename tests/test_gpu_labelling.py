"""GPU parity of the labelling score (per-element F1 of section 5.2) against
the CPU oracle.  The counts are integers, so the class map is compared exactly
and every score to 1e-12."""
import numpy as np
import pytest
import torch

import oracle
from oracle import labelling as LB
from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError

pytestmark = pytest.mark.gpu


def _check(res, ref, C):
    assert res["map"] == ref["map"].tolist()
    np.testing.assert_allclose(res["precision"], ref["precision"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(res["recall"], ref["recall"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(res["f1"], ref["f1"], rtol=0, atol=1e-12)
    assert abs(res["macro_f1"] - ref["macro_f1"]) < 1e-12


@pytest.mark.parametrize("case", ["four_regimes", "regimes5_n100000"])
def test_label_f1_matches_oracle(case):
    if case == "four_regimes":
        S = synth.four_regimes(1)
        m, l, K = 100, 50, 4
    else:
        S = synth.regime_series(100_000, 2, synth.SHAPES5)
        m, l, K = 256, 128, 5
    C = int(S.labels.max()) + 1
    T = torch.from_numpy(S.x).cuda()
    out = api.snippets(T, m, l, K, owner=True)
    owner = out["owner"]
    truth = torch.from_numpy(S.labels.astype(np.int32)).cuda()
    res = api.label_f1(owner, truth, m, K, C)
    ref = LB.label_f1(owner.cpu().numpy(), S.labels, m, K, C)
    _check(res, ref, C)
    print(f"{case}: macro F1 {res['macro_f1']:.4f}, map {res['map']}", flush=True)
    if case == "four_regimes":
        # the whole chain from the oracle's own profiles gives the same labelling
        ref_chain = oracle.snippets(S.x, m, l, K)
        r2 = LB.label_f1(ref_chain["owner"], S.labels, m, K, C)
        assert abs(r2["macro_f1"] - res["macro_f1"]) < 1e-3


def test_label_f1_wide_table_and_errors():
    # K*C beyond the LDS table: counts go straight to device memory
    rng = np.random.default_rng(3)
    n, m, K, C = 5000, 50, 3, 3000
    owner_np = rng.integers(0, K, n - m + 1).astype(np.int32)
    truth_np = rng.integers(0, 7, n).astype(np.int32)
    owner = torch.from_numpy(owner_np).cuda()
    truth = torch.from_numpy(truth_np).cuda()
    res = api.label_f1(owner, truth, m, K, C)
    _check(res, LB.label_f1(owner_np, truth_np, m, K, C), C)
    bad = truth.clone()
    bad[17] = C  # outside [0, C)
    with pytest.raises(PstError):
        api.label_f1(owner, bad, m, K, C)
    res2 = api.label_f1(owner, truth, m, K, C)   # the context still works
    assert res2["map"] == res["map"]
