"""Precision study on the 10^6-point random walk with planted periodic regimes
(m=512, l=256, k=52): profile error of the FP32 recurrence against the FP64
oracle, for the default anchoring (an FP64 anchor at the first cell of every
diagonal of a sub-tile, so at most w-1 = 256 FP32 steps) and for extra FP64
re-anchors every R rows, R in {128, 32} and the study's {256, 1024, 4096}.
With w = 257 rows per sub-tile, R = 256 adds one re-anchor (row 256) and
R >= 1024 none: those profiles are bit-identical to the default's.  Errors
are measured on sampled profile entries, each computed by the oracle on its
own."""
import math
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13680_amd import _lib, api, synth

pytestmark = pytest.mark.gpu


def test_precision_walk_n1000000():
    x = synth.long_walk(1_000_000, 4).x
    m, l, k = 512, 256, 52
    T = torch.from_numpy(x).cuda()
    nseg, Nm = len(x) // m, len(x) - m + 1
    rng = np.random.default_rng(7)
    pairs = [(int(rng.integers(nseg)), int(rng.integers(Nm))) for _ in range(120)]
    pairs += [(s, s * m) for s in range(0, nseg, 150)]
    # windows inside planted regimes (50 000 + 100 000 r) against segments there
    pairs += [(int((50_000 + 100_000 * r) // m) + 2, 50_000 + 100_000 * r + 1000 + 37 * r) for r in range(10)]
    ref = oracle.mpdist_pairs_local(x, m, l, k, pairs)
    ctx = api.context(0)
    rows = []
    D0 = None
    for R in (0, 4096, 1024, 256, 128, 32):
        ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_ANCHOR_EVERY, R))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D, _ = api.profile_set(T, m, l, k, ctx=ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if R == 0:
            D0 = D
        elif R >= 1024:
            assert torch.equal(D, D0), R          # no re-anchor inside a sub-tile
        idx = torch.from_numpy(np.array(pairs).T.copy()).cuda()
        got = D[idx[0], idx[1]].cpu().numpy().astype(np.float64)
        if R != 0:
            del D
        e = np.abs(got ** 2 - ref ** 2) / (4 * l)
        mask = ref >= 0.1 * math.sqrt(l)
        rel = np.abs(got - ref)[mask] / ref[mask]
        rows.append((R, dt, e.max(), e.mean(), rel.max(), rel.mean()))
    del D0
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_ANCHOR_EVERY, 0))
    print("\nR(0=per sub-tile)  seconds  max_e  mean_e  max_rel  mean_rel")
    for r in rows:
        print("%5d %8.2f %9.3g %9.3g %9.3g %9.3g" % r, flush=True)
    for R, dt, emax, emean, rmax, rmean in rows:
        assert emax <= 1e-4 and rmax <= 1e-4, (R, emax, rmax)
