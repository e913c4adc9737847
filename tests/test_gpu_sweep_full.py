"""The length sweep at full size (the 250 000-point six-shape series of the
sweep benchmark, l = m/2, K = 6, over all fifteen of its lengths, m = 64 ..
512 step 32, or over twelve of them, m = 64 .. 288 and 416 .. 512, or ten,
m = 64 .. 288 and 480, 512, or five, m = 64, 128, 224, 480, 512) against the
oracle's stored results (tests/golden/sweep_regimes6_n250000_sweep.json,
..._sweep12.json, ..._sweep10.json or ..._sweep5.json, whichever is the
longest there, written by tests/golden/make_golden.py from oracle/ only).

Per length, the GPU's snippets are checked step by step against the oracle's
pick and runner-up: while the GPU's picks equal the oracle's, the two
candidates' areas on the GPU's own profiles (FP64 sums) differ from the
oracle's stored areas by e_b and e_r, and the GPU must make the oracle's pick
wherever the oracle's margin exceeds 4 (e_b + e_r) (the oracle's full profile
set, needed for the exact bound of tests/greedy_bounds.py, is not stored at
this size).  ProfileArea equals an FP64 recompute from the GPU's profiles.  The
eq. 18 scores match to 1e-3 relative and the batched sweep picks the
oracle's m_best wherever the two best scores are further apart than that."""
import json
import os

import numpy as np
import pytest
import torch

from greedy_bounds import areas_from_profiles
from paper_2401_13680_amd import api, synth

pytestmark = pytest.mark.gpu
_G = os.path.join(os.path.dirname(__file__), "golden")
# the longest list of lengths that has been written
GOLD = next((os.path.join(_G, f) for f in ("sweep_regimes6_n250000_sweep.json",
                                           "sweep_regimes6_n250000_sweep12.json",
                                           "sweep_regimes6_n250000_sweep10.json",
                                           "sweep_regimes6_n250000_sweep5.json")
             if os.path.exists(os.path.join(_G, f))), os.path.join(_G, "sweep_regimes6_n250000_sweep5.json"))


def _area(M, row):
    return float(np.sum(np.minimum(M, row)))


@pytest.mark.skipif(not os.path.exists(GOLD), reason="oracle sweep results not generated")
def test_sweep_n250000_matches_oracle():
    gold = json.load(open(GOLD))
    x = synth.regime_series(250_000, 3, synth.SHAPES6).x
    T = torch.from_numpy(x).cuda()
    K = gold["K"]
    print(f"sweep n=250000: {len(gold['m_list'])} lengths", flush=True)
    sw = api.select_length(T, gold["m_list"], K)
    for a, b in zip(sw["scores"], gold["scores"]):
        assert abs(a - b) <= 1e-3 * abs(b), (a, b)
    s = sorted(gold["scores"], reverse=True)
    if s[0] - s[1] > 2e-3 * s[0]:
        assert sw["m_best"] == gold["m_best"]
    for g in gold["lengths"]:
        m, l = g["m"], g["l"]
        r = api.snippets(T, m, l, K, profiles=True)
        by_rank = sorted(r["records"], key=lambda q: q["greedy_rank"])
        picks = [rec["segment"] for rec in by_rank]
        np.testing.assert_allclose([rec["area_after"] for rec in by_rank],
                                   areas_from_profiles(r["profiles"].cpu().numpy()), rtol=1e-12)
        D, _ = api.profile_set(T, m, l)
        rows = sorted(set(picks) | set(g["picks"]) | {q for q in g["runners"] if q is not None})
        Dg = {s_: row for s_, row in zip(rows, D[rows].cpu().numpy().astype(np.float64))}
        del D
        M = np.full(len(x) - m + 1, np.inf)
        for t, c in enumerate(picks):
            b, rr = g["picks"][t], g["runners"][t]
            if picks[:t] == g["picks"][:t]:
                # same curve on both sides: the oracle's best and runner-up
                # areas against the same rows' areas on the GPU's profiles
                ab, ar = g["areas"][t], g["areas"][t] + g["margins"][t]
                eb, er = abs(_area(M, Dg[b]) - ab), abs(_area(M, Dg[rr]) - ar)
                print(f"m={m} step {t}: oracle {b} margin {g['margins'][t]:.6g} gpu {c} "
                      f"area errors {eb:.3g} {er:.3g}", flush=True)
                if g["margins"][t] > 4 * (eb + er):
                    assert c == b, (m, t, c, b)
            M = np.minimum(M, Dg[c])
