"""Every tile geometry the profile kernel can run (workgroup size, diagonals
per thread, rows per chunk, selection threads, sub-tile width), installed one
at a time, against the FP64 oracle: profiles within the stated tolerance and
snippets margin-aware equal to the oracle's; and the tuner, which times the
candidates on a series and installs the fastest, remembering it in the cache
file.  The built-in geometry is restored afterwards."""
import numpy as np
import pytest
import torch

import oracle
from greedy_bounds import areas_from_profiles, check_greedy
from paper_2401_13680_amd import api, synth

pytestmark = pytest.mark.gpu
TOL = 1e-4

CASES = [
    # name, series, m, l, K
    ("w51", lambda: synth.four_regimes(1).x, 100, 50, 3),
    ("w129", lambda: synth.regime_series(9000, 61, len_range=(1000, 3000)).x, 256, 128, 3),
    ("w257", lambda: synth.regime_series(9000, 62, len_range=(1000, 3000)).x, 512, 256, 2),
    ("w513", lambda: synth.regime_series(9000, 63, len_range=(1000, 3000)).x, 1024, 512, 2),
]


@pytest.mark.parametrize("name,gen,m,l,K", CASES, ids=[c[0] for c in CASES])
def test_every_geometry_matches_oracle(name, gen, m, l, K):
    x = gen()
    w = m - l + 1
    T = torch.from_numpy(x).cuda()
    Dr = oracle.profile_set(x, m, l)
    codes = api.geometry_candidates(w)
    assert api.geometry(w) in codes
    try:
        for code in codes:
            print(f"{name}: geometry {code:#x} {api.decode_geometry(code)}", flush=True)
            api.set_geometry(w, code)
            assert api.geometry(w) == code
            D, _ = api.profile_set(T, m, l)
            Dg = D.cpu().numpy().astype(np.float64)
            e = np.abs(Dg ** 2 - Dr ** 2).max() / (4 * l)
            assert e <= TOL, (code, e)
            r = api.snippets(T, m, l, K, profiles=True)
            by_rank = sorted(r["records"], key=lambda q: q["greedy_rank"])
            picks = [q["segment"] for q in by_rank]
            check_greedy(picks, {s: Dg[s] for s in range(len(Dg))}, {s: Dr[s] for s in range(len(Dr))},
                         list(range(len(Dr))), f"{name} {code:#x}")
            np.testing.assert_allclose([q["area_after"] for q in by_rank],
                                       areas_from_profiles(r["profiles"].cpu().numpy()), rtol=1e-12)
    finally:
        api.set_geometry(w, 0)


def test_tuner_installs_a_candidate_and_remembers_it(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PST_AUTOTUNE_CACHE", str(cache))
    x = synth.regime_series(20_000, 64, len_range=(1000, 3000)).x
    T = torch.from_numpy(x).cuda()
    m, l = 200, 100
    w = m - l + 1
    try:
        code, ms = api.tune_geometry(T, m, l)
        print(f"tuned w={w}: {code:#x} {api.decode_geometry(code)} {ms:.3f} ms", flush=True)
        assert code in api.geometry_candidates(w) and ms > 0
        assert api.geometry(w) == code
        lines = [ln.split() for ln in cache.read_text().splitlines() if ln.startswith("geo ")]
        assert any(int(f[2]) == w and int(f[3]) == code for f in lines)
        # the remembered choice comes back without timing
        api.set_geometry(w, 0)
        code2, _ = api.tune_geometry(T, m, l)
        assert code2 == code and api.geometry(w) == code
        D, _ = api.profile_set(T, m, l)
        Dr = oracle.profile_set(x, m, l, segments=[0, 7, 50])
        e = np.abs(D.cpu().numpy()[[0, 7, 50]].astype(np.float64) ** 2 - Dr ** 2).max() / (4 * l)
        assert e <= TOL
    finally:
        api.set_geometry(w, 0)


def test_sweep_with_tuned_geometries_matches_oracle():
    """The batched sweep with every length's geometry tuned first: scores
    within 1e-3 of the oracle's and the oracle's m_best."""
    x = synth.regime_series(6000, 65, len_range=(600, 1500)).x
    ms = [40, 64, 200, 380]
    T = torch.from_numpy(x).cuda()
    ws = [m - m // 2 + 1 for m in ms]
    try:
        r = api.select_length(T, ms, 3, tune_geometry=True)
        print("tuned:", {w: hex(api.geometry(w)) for w in ws}, flush=True)
        ref = oracle.select_length(x, ms, 3)
        for a, b in zip(r["scores"], ref["scores"]):
            assert abs(a - b) <= 1e-3 * max(1.0, abs(b))
        assert r["m_best"] == ref["m_best"]
    finally:
        for w in ws:
            api.set_geometry(w, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("graph", [False, True])
def test_sweep_in_one_launch_matches_oracle(graph):
    """Every length of the sweep in one launch, in the widest length's
    geometry (lengths of several workgroup shapes): scores within 1e-3 of the
    oracle's, its m_best, and scores within 1e-4 of the per-shape launches'."""
    x = synth.regime_series(6000, 66, len_range=(600, 1500)).x
    ms = [24, 64, 200, 600]
    T = torch.from_numpy(x).cuda()
    shapes = {(api.geometry(m - m // 2 + 1) >> 24) & 15 for m in ms}
    assert len(shapes) > 1
    r = api.select_length(T, ms, 3, one_launch=True, graph=graph)
    split = api.select_length(T, ms, 3, one_launch=False, graph=graph)
    ref = oracle.select_length(x, ms, 3)
    for a, b in zip(r["scores"], ref["scores"]):
        assert abs(a - b) <= 1e-3 * max(1.0, abs(b))
    assert r["m_best"] == ref["m_best"]
    for a, b in zip(r["scores"], split["scores"]):
        assert abs(a - b) <= 1e-4 * max(1.0, abs(b))
