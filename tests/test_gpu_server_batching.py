"""Continuous batching in the request server: requests of one tile geometry
that are ready together run their profiles in one persistent launch.  Every
result must equal the same request run alone with pst_snippets, whether the
series came from host memory or from a device tensor."""
import pytest
import torch

from paper_2401_13680_amd import api, synth

pytestmark = pytest.mark.gpu


def test_batched_requests_equal_alone():
    specs = [(n, m, K, 40 + i) for i, (n, m, K) in enumerate(
        [(6_000, 64, 3), (9_000, 96, 4), (12_000, 128, 3), (5_000, 64, 5), (15_000, 96, 3),
         (7_000, 128, 4), (20_000, 64, 3), (8_000, 96, 5), (11_000, 128, 3), (6_500, 64, 4)])]
    xs = [synth.regime_series(n, seed, len_range=(800, 3000)).x for n, _, _, seed in specs]
    print(f"server batching: {len(specs)} requests, m in (64, 96, 128)", flush=True)
    srv = api.Server(0, hbm_budget_bytes=16 << 30, max_slots=16)
    # every other series is handed over as a device tensor
    ins = [torch.from_numpy(x).cuda() if i % 2 else x for i, x in enumerate(xs)]
    torch.cuda.synchronize()
    tickets = [srv.submit(s, m, m // 2, K) for s, (n, m, K, _) in zip(ins, specs)]
    srv.drain()
    got = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"batches: {st['batches']}", flush=True)
    assert st["batches"] < len(specs)
    for g, x, (n, m, K, _) in zip(got, xs, specs):
        assert g["status"] == 0
        alone = api.snippets(torch.from_numpy(x).cuda(), m, m // 2, K)
        assert g["records"] == alone["records"], (n, m, K)
