"""GPU parity: the HIP library against the FP64 CPU oracle on seeded inputs.

Tolerance (stated for FP32 profiles against FP64): for every profile entry
    e = |d_gpu^2 - d_ref^2| / (4 l) <= 1e-4
(relative to the range [0, 4l] of d^2; equivalent to |delta rho| <= 2e-4), and
    |d_gpu - d_ref| / d_ref <= 1e-4   wherever d_ref >= 0.1 sqrt(l)
(a plain relative bound where it is meaningful: near d = 0 the square root
turns one FP32 rounding of rho into ~sqrt(l * 1e-7)).  Snippet indices,
greedy order and neighbour counts are compared exactly.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from greedy_bounds import areas_from_profiles, check_greedy
from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError

pytestmark = pytest.mark.gpu
TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def profile_errors(gpu, ref, l):
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    e = np.abs(g * g - r * r) / (4.0 * l)
    mask = r >= 0.1 * math.sqrt(l)
    rel = np.abs(g - r)[mask] / r[mask] if mask.any() else np.zeros(1)
    return float(e.max()), float(rel.max())


def assert_profiles_close(gpu, ref, l, what=""):
    e, rel = profile_errors(gpu, ref, l)
    print(f"{what}: max e={e:.3g} max rel={rel:.3g}", flush=True)
    assert e <= TOL, (what, e)
    assert rel <= TOL, (what, rel)


CASES = [
    # name, series, m, l, k
    ("four_regimes", lambda: synth.four_regimes(1).x, 100, 50, 10),
    ("ragged_tiles", lambda: synth.regime_series(3100, 21, len_range=(300, 900)).x, 40, 20, 0),
    ("l_eq_m", lambda: synth.random_tiny(1500, 3), 30, 30, 3),
    ("l_eq_2", lambda: synth.random_tiny(1200, 4), 24, 2, 0),
    ("k_over_2w", lambda: synth.random_tiny(900, 5), 20, 18, 10),
    ("n_not_multiple", lambda: synth.regime_series(2050, 6, len_range=(200, 600)).x, 64, 32, 0),
    ("wide_w", lambda: synth.regime_series(3000, 7, len_range=(300, 900)).x, 256, 32, 0),
    ("random_walk", lambda: np.cumsum(np.random.default_rng(8).normal(size=2500)) + 500.0, 50, 25, 0),
    # every workgroup shape of the profile kernel: 256 threads with 6 diagonals
    # per thread; 512 threads with 256 blocks per tile, 5 or 6 diagonals, 4 or
    # 8 rows per chunk, 1984 or 992 windows per sub-tile; the largest w
    ("w160_v6", lambda: synth.regime_series(3000, 22, len_range=(300, 900)).x, 320, 161, 0),
    ("w270", lambda: synth.regime_series(3200, 23, len_range=(300, 900)).x, 400, 131, 0),
    ("w400", lambda: synth.regime_series(3000, 24, len_range=(300, 900)).x, 500, 101, 0),
    ("w700", lambda: synth.regime_series(3000, 25, len_range=(300, 900)).x, 800, 101, 0),
    ("w_max_1025", lambda: synth.regime_series(2500, 26, len_range=(300, 900)).x, 1100, 76, 0),
]


@pytest.mark.parametrize("name,gen,m,l,k", CASES, ids=[c[0] for c in CASES])
def test_profile_set_matches_oracle(name, gen, m, l, k):
    x = gen()
    print(f"case {name}: n={len(x)} m={m} l={l} k={k}", flush=True)
    D, dmax = api.profile_set(dev(x), m, l, k)
    torch.cuda.synchronize()
    Dref = oracle.profile_set(x, m, l, k if k > 0 else None)
    assert tuple(D.shape) == Dref.shape
    Dg = D.cpu().numpy()
    assert_profiles_close(Dg, Dref, l, name)
    assert float(dmax.item()) == float(Dg.max())


def test_query_profile_matches_oracle():
    x = synth.four_regimes(1).x
    q = synth.random_tiny(100, 12)
    out = api.mpdist_profile(dev(x), dev(q), 50, 10)
    ref = oracle.mpd(q, x, 50, 10)
    assert_profiles_close(out.cpu().numpy(), ref, 50, "query")
    # a window of T as the query scores zero at its own position
    out2 = api.mpdist_profile(dev(x), dev(x[700:800]), 50, 10).cpu().numpy()
    assert out2[700] < math.sqrt(2 * 50 * 8 * 2 ** -23)


def test_snippets_four_regimes_match_golden():
    """Snippets of the 2000-point four-regime series against the oracle, step by
    step with the margin-aware bound (tests/greedy_bounds.py): the GPU's pick
    must be the oracle's wherever the oracle's margin exceeds the bound that the
    profile differences put on the areas.  ProfileArea after each pick equals
    an FP64 recompute from the GPU's own returned profiles."""
    gold = json.load(open(os.path.join(GOLDEN, "snippets_four_regimes_n2000.json")))
    x = synth.four_regimes(1).x
    m, l, k, K = gold["m"], gold["l"], gold["k"], gold["K"]
    r = api.snippets(dev(x), m, l, K, k, profiles=True, owner=True)
    D, _ = api.profile_set(dev(x), m, l, k)
    Dg = D.cpu().numpy().astype(np.float64)
    Dr = oracle.profile_set(x, m, l, k)
    by_rank = sorted(r["records"], key=lambda rec: rec["greedy_rank"])
    picks = [rec["segment"] for rec in by_rank]
    res = check_greedy(picks, {s: Dg[s] for s in range(len(Dg))}, {s: Dr[s] for s in range(len(Dr))},
                       list(range(len(Dr))), "four_regimes")
    for (margin, B, _), gm in zip(res, gold["margins"]):
        assert margin == pytest.approx(gm, rel=1e-9)
    prof = r["profiles"].cpu().numpy()
    np.testing.assert_array_equal(prof, D.cpu().numpy()[picks])
    np.testing.assert_allclose([rec["area_after"] for rec in by_rank], areas_from_profiles(prof), rtol=1e-12)
    if picks == gold["picks"]:
        for a, b in zip(r["records"], gold["records"]):
            assert (a["segment"], a["greedy_rank"], a["frac"]) == (b["segment"], b["greedy_rank"], b["frac"])
        own = r["owner"].cpu().numpy()
        counts = [int(np.count_nonzero(own == p)) for p in range(K)]
        assert counts == gold["counts"]
    assert abs(r["dmax"] - gold["dmax"]) <= 1e-4 * gold["dmax"]


def test_planted_repeats_bit_identical_and_recovered():
    m, l = 64, 32
    x, order = synth.planted_motifs(m, 3, [3, 2, 4], seed=1)
    D, _ = api.profile_set(dev(x), m, l)
    Dg = D.cpu().numpy()
    for s in range(len(order)):
        for t in range(len(order)):
            if order[s] == order[t]:
                assert np.array_equal(Dg[s], Dg[t])            # bitwise identical rows
                assert Dg[s, t * m] <= math.sqrt(2 * l * 8 * 2 ** -23)
    r = api.snippets(dev(x), m, l, 3)
    first = {int(np.flatnonzero(order == mid)[0]) for mid in range(3)}
    assert {rec["segment"] for rec in r["records"]} == first
    ref = oracle.snippets(x, m, l, 3)
    assert [rec["segment"] for rec in r["records"]] == [rec["segment"] for rec in ref["records"]]


def test_constant_windows_match_oracle():
    rng = np.random.default_rng(0)
    x = np.concatenate([np.full(300, 2.0), rng.normal(size=300), np.full(300, -1.0),
                        np.sin(np.arange(300) / 7.0)])
    D, _ = api.profile_set(dev(x), 40, 20)
    ref = oracle.profile_set(x, 40, 20)
    assert_profiles_close(D.cpu().numpy(), ref, 20, "constant")


def test_select_length_matches_oracle():
    x = synth.regime_series(4000, 9, len_range=(500, 1500)).x
    ms = [40, 64, 100]
    r = api.select_length(dev(x), ms, 3, profiles=True, owner=True)
    ref = oracle.select_length(x, ms, 3)
    print("scores gpu", r["scores"], "oracle", ref["scores"], flush=True)
    for a, b in zip(r["scores"], ref["scores"]):
        assert abs(a - b) <= 1e-3 * max(1.0, abs(b))
    assert r["m_best"] == ref["m_best"]
    best = ms.index(ref["m_best"])
    assert [rec["segment"] for rec in r["records"]] == \
        [rec["segment"] for rec in ref["results"][best]["records"]]
    assert r["profiles"].shape == (3, len(x) - ref["m_best"] + 1)


def test_errors_are_reported_and_context_survives():
    x = synth.four_regimes(1).x
    with pytest.raises(PstError) as ei:
        api.snippets(dev(x), 100, 50, 21)
    assert ei.value.code == -1
    with pytest.raises(PstError):
        api.profile_set(dev(x), 100, 101)
    bad = x.copy()
    bad[1234] = np.nan
    with pytest.raises(PstError) as ei:
        api.profile_set(dev(bad), 100, 50)
    assert "non-finite" in str(ei.value)
    D, _ = api.profile_set(dev(x), 100, 50)      # the context still works
    assert torch.isfinite(D).all()


def test_deterministic():
    x = synth.regime_series(5000, 10, len_range=(500, 1500)).x
    a, _ = api.profile_set(dev(x), 64, 32)
    b, _ = api.profile_set(dev(x), 64, 32)
    assert torch.equal(a, b)


def test_full_size_sampled_and_snippets():
    """The 100k-point, m=256 workload at full size: sampled profile entries
    (one window of every segment and more) against the oracle one by one, the
    whole rows of the picks and runners-up against the oracle's rows, and the
    snippets against the stored oracle result with the margin-aware bound,
    computed from those rows."""
    gold = json.load(open(os.path.join(GOLDEN, "snippets_regimes5_n100000.json")))
    x = synth.regime_series(100_000, 2, synth.SHAPES5).x
    m, l, k, K = gold["m"], gold["l"], gold["k"], gold["K"]
    D, dmax = api.profile_set(dev(x), m, l, k)
    rng = np.random.default_rng(0)
    nseg, Nm = D.shape
    pairs = [(int(rng.integers(nseg)), int(rng.integers(Nm))) for _ in range(60)]
    pairs += [(s, s * m) for s in range(0, nseg, 97)] + [(nseg - 1, Nm - 1), (0, 0)]
    pairs += [(s, int(rng.integers(Nm))) for s in range(nseg)]  # one window of every segment
    ref = oracle.mpdist_samples(x, m, l, k, pairs)
    Dg = D.cpu().numpy()
    got = np.array([Dg[s, j] for s, j in pairs])
    assert_profiles_close(got, ref, l, "full-size samples")
    assert abs(float(dmax.item()) - gold["dmax"]) <= 1e-4 * gold["dmax"]
    r = api.snippets(dev(x), m, l, K, k, profiles=True)
    by_rank = sorted(r["records"], key=lambda rec: rec["greedy_rank"])
    picks = [rec["segment"] for rec in by_rank]
    cands = sorted(set(gold["picks"]) | set(gold["runners"]) | set(picks))
    print(f"full size: oracle rows of segments {cands}", flush=True)
    Dr = oracle.profile_set(x, m, l, k, segments=cands)
    # those whole rows too: every window of the series, entry by entry
    assert_profiles_close(Dg[cands].astype(np.float64), Dr, l, "full-size oracle rows")
    rows_r = {s: Dr[i] for i, s in enumerate(cands)}
    rows_g = {s: Dg[s].astype(np.float64) for s in cands}
    res = check_greedy(picks, rows_g, rows_r, cands, "regimes5_n100000")
    assert picks == gold["picks"] or not all(eq for _, _, eq in res)
    prof = r["profiles"].cpu().numpy()
    np.testing.assert_allclose([rec["area_after"] for rec in by_rank], areas_from_profiles(prof), rtol=1e-12)
    if picks == gold["picks"]:
        for a, b in zip(r["records"], gold["records"]):
            assert a["segment"] == b["segment"] and abs(a["frac"] - b["frac"]) <= 1e-3


def _sweep_key(r):
    return (r["m_best"], list(r["scores"]), [(x["segment"], x["greedy_rank"], x["frac"], x["area_after"])
                                           for x in r["records"]])


def test_sweep_batched_graph_equals_plain_and_oracle():
    """All candidate lengths in one launch (eager and graph-captured) give the
    same scores and snippets as the one-length-at-a-time path, bit for bit, and
    match the oracle."""
    x = synth.regime_series(6000, 13, len_range=(600, 1500)).x
    ms = [40, 56, 72, 88]
    T = dev(x)
    plain = api.select_length(T, ms, 3, batched=False)
    eager = api.select_length(T, ms, 3, batched=True, graph=False)
    assert _sweep_key(eager) == _sweep_key(plain)
    ref = oracle.select_length(x, ms, 3)
    for a, b in zip(eager["scores"], ref["scores"]):
        assert abs(a - b) <= 1e-3 * max(1.0, abs(b))
    assert eager["m_best"] == ref["m_best"]
    # graph replays, with eager work and synchronisations in between
    for rep in range(3):
        g = api.select_length(T, ms, 3, batched=True, graph=True, profiles=True, owner=True)
        assert _sweep_key(g) == _sweep_key(eager), rep
        D, _ = api.profile_set(T, 64, 32)        # unrelated eager work
        torch.cuda.synchronize()
    best = ms.index(g["m_best"])
    Dref = oracle.profile_set(x, g["m_best"], g["m_best"] // 2)
    picks = [rec["segment"] for rec in sorted(g["records"], key=lambda r: r["greedy_rank"])]
    assert_profiles_close(g["profiles"].cpu().numpy(), Dref[picks], g["m_best"] // 2, "sweep profiles")


def test_sweep_across_workgroup_shapes():
    """Lengths whose profile kernels use different workgroup shapes (w = 25
    and 33 with 256 threads, w = 191 and 257 with 512) run as two launches in
    the batched sweep: same scores and snippets as one length at a time, and
    the oracle's choice."""
    x = synth.regime_series(4000, 15, len_range=(600, 1500)).x
    ms = [48, 64, 380, 512]
    T = dev(x)
    print("sweep: n=4000 m in {48, 64, 380, 512}", flush=True)
    plain = api.select_length(T, ms, 2, batched=False)
    for graph in (False, True):
        b = api.select_length(T, ms, 2, batched=True, graph=graph)
        assert _sweep_key(b) == _sweep_key(plain), graph
    ref = oracle.select_length(x, ms, 2)
    for a, r in zip(plain["scores"], ref["scores"]):
        assert abs(a - r) <= 1e-3 * max(1.0, abs(r))
    assert plain["m_best"] == ref["m_best"]


def test_sweep_autotune_same_result(tmp_path, monkeypatch):
    monkeypatch.setenv("PST_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    x = synth.regime_series(5000, 14, len_range=(500, 1500)).x
    ms = [48, 64, 80]
    T = dev(x)
    a = api.select_length(T, ms, 2, autotune=False)
    b = api.select_length(T, ms, 2, autotune=True)
    assert _sweep_key(a) == _sweep_key(b)


_TUNED_SWEEP = (
    "import json, torch\n"
    "from paper_2401_13680_amd import api, synth\n"
    "x = synth.regime_series(5000, 14, len_range=(500, 1500)).x\n"
    "r = api.select_length(torch.from_numpy(x).cuda(), [48, 64, 80], 2, autotune=True)\n"
    "print(json.dumps([r['m_best'], list(r['scores']),\n"
    "                  [(q['segment'], q['greedy_rank'], q['area_after']) for q in r['records']]]))\n")


def test_cached_grid_past_the_workspace_is_clamped(tmp_path):
    """A line of the tuning cache file may come from another build: a cached
    persistent grid larger than the sweep's workspace has scratch slots for is
    clamped to the plan's grid.  The second process takes the cached line
    (it appends none) and returns the first one's result exactly."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, PST_AUTOTUNE_CACHE=str(cache))

    def run():
        p = subprocess.run([sys.executable, "-c", _TUNED_SWEEP], cwd=root, env=env,
                           capture_output=True, text=True, timeout=300)
        assert p.returncode == 0, p.stderr[-2000:]
        return json.loads(p.stdout.strip().splitlines()[-1])

    first = run()
    lines = cache.read_text().splitlines()
    grid_lines = [q for q in lines if q.split()[0] != "geo"]
    assert grid_lines, lines
    # "arch wmax tiles_log2 grid dynamic ms": the grid far past any workspace
    cache.write_text("".join(" ".join(f[:3] + ["1000000"] + f[4:]) + "\n" if f[0] != "geo" else q + "\n"
                             for q in lines for f in [q.split()]))
    second = run()
    assert len(cache.read_text().splitlines()) == len(lines)
    assert second == first


def test_server_results_equal_alone_and_in_mix():
    """Requests of different n, m and K submitted together overlap on the
    device; each result equals the same request run alone with pst_snippets,
    and a request with a non-finite value fails alone."""
    specs = [(20_000, 64, 3, 31), (50_000, 256, 4, 32), (8_000, 128, 5, 33),
             (30_000, 512, 3, 34), (12_000, 96, 4, 35), (40_000, 1024, 3, 36)]
    xs = [synth.regime_series(n, seed, len_range=(1000, 4000)).x for n, _, _, seed in specs]
    srv = api.Server(0, hbm_budget_bytes=8 << 30, max_slots=4)
    tickets = [srv.submit(x, m, m // 2, K) for x, (n, m, K, _) in zip(xs, specs)]
    bad = xs[2].copy()
    bad[100] = np.inf
    tbad = srv.submit(bad, 128, 64, 5)
    srv.drain()
    got = [srv.poll(t) for t in tickets]
    rb = srv.poll(tbad)
    assert rb["status"] == -1
    st = srv.stats()
    srv.close()
    for g, x, (n, m, K, _) in zip(got, xs, specs):
        assert g["status"] == 0 and g["latency_ms"] > 0
        alone = api.snippets(dev(x), m, m // 2, K)
        assert g["records"] == alone["records"], (n, m, K)
    assert st["completed"] == len(specs) + 1 and st["active"] == 0


def test_reanchor_option_keeps_parity():
    x = synth.regime_series(4000, 19, len_range=(400, 1200)).x
    ctx = api.context(0)
    ref = oracle.profile_set(x, 80, 40)
    for R in (7, 16):
        ctx.check(ctx.L.pst_set_option(ctx.h, 6, R))
        D, _ = api.profile_set(dev(x), 80, 40, ctx=ctx)
        assert_profiles_close(D.cpu().numpy(), ref, 40, f"R={R}")
    ctx.check(ctx.L.pst_set_option(ctx.h, 6, 0))
