"""The server's shortest-predicted-first admission (section 4.2's run-time
prediction applied to one GPU's queue): every request's result equals the
same request run alone, whatever the order, and the model learns from the
completed requests."""
import numpy as np
import pytest
import torch

from paper_2401_13680_amd import api, synth
from paper_2401_13680_amd._lib import PstError

pytestmark = pytest.mark.gpu


def test_shortest_predicted_first_results_equal_alone():
    specs = [(40_000, 512, 3, 41), (6_000, 64, 4, 42), (25_000, 256, 5, 43), (9_000, 96, 3, 44),
             (30_000, 128, 4, 45), (7_000, 192, 3, 46), (15_000, 64, 5, 47), (11_000, 320, 4, 48),
             (5_000, 100, 3, 49), (20_000, 384, 3, 50)]
    print("server policy: 10 requests, 2 slots, shortest predicted first", flush=True)
    xs = [synth.regime_series(n, seed, len_range=(1000, 4000)).x for n, _, _, seed in specs]
    seed = api.RuntimeModel(2)
    for n, m, _, _ in specs[:4]:
        seed.observe(n, m, m // 2, 1e-8 * (n // m) * (m - m // 2 + 1) * (n - m // 2 + 1))
    seed.fit()
    srv = api.Server(0, hbm_budget_bytes=8 << 30, max_slots=2)
    srv.set_policy(api.Server.SHORTEST_PREDICTED, seed)
    tickets = [srv.submit(x, m, m // 2, K) for x, (n, m, K, _) in zip(xs, specs)]
    srv.drain()
    got = [srv.poll(t) for t in tickets]
    # a second round without a seed model (cell counts until the first fit)
    srv.set_policy(api.Server.SHORTEST_PREDICTED)
    t2 = [srv.submit(x, m, m // 2, K) for x, (n, m, K, _) in zip(xs[:4], specs[:4])]
    srv.drain()
    got2 = [srv.poll(t) for t in t2]
    st = srv.stats()
    with pytest.raises(PstError):
        srv.set_policy(7)
    srv.set_policy(api.Server.ARRIVAL)
    srv.close()
    for g, x, (n, m, K, _) in zip(got + got2, xs + xs[:4], specs + specs[:4]):
        assert g["status"] == 0 and g["latency_ms"] > 0
        alone = api.snippets(torch.from_numpy(x).cuda(), m, m // 2, K)
        assert g["records"] == alone["records"], (n, m, K)
    assert st["completed"] == len(specs) + 4 and st["active"] == 0
