"""The allocation-free query profile (pst_mpdist_profile_noalloc) against
pst_mpdist_profile, through the C ABI: two calls in a row, the second on a
smaller input, each equal to the workspace-taking entry point's result (the
tile arithmetic does not depend on the grid, so bit for bit), and within the
parity tolerance of the oracle; an input too large for the fixed scratch is
refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13680_amd import _lib, api, synth

pytestmark = pytest.mark.gpu


def _noalloc(ctx, T, Q, l, k):
    n, m = T.numel(), Q.numel()
    out = torch.empty(n - m + 1, dtype=torch.float32, device=T.device)
    rc = ctx.L.pst_mpdist_profile_noalloc(ctx.h, ctypes.c_void_p(T.data_ptr()), n, ctypes.c_void_p(Q.data_ptr()),
                                          m, l, k, ctypes.c_void_p(out.data_ptr()))
    return rc, out


def test_noalloc_profile_equals_workspace_path_twice():
    ctx = api.context(0)
    cases = [(synth.regime_series(30_000, 41, len_range=(2000, 6000)).x, 256, 128, 26, 3000),
             (synth.regime_series(5_000, 42, len_range=(500, 1500)).x, 100, 50, 10, 700)]
    for x, m, l, k, q0 in cases:
        print(f"noalloc: n={len(x)} m={m} l={l} k={k}", flush=True)
        T = torch.from_numpy(x).cuda()
        Q = T[q0:q0 + m].clone()
        rc, got = _noalloc(ctx, T, Q, l, k)
        assert rc == 0, ctx.L.pst_last_error(ctx.h).decode()
        want = api.mpdist_profile(T, Q, l, k, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        ref = oracle.mpd(x[q0:q0 + m], x, l, k)
        e = np.abs(got.cpu().numpy().astype(np.float64) ** 2 - ref ** 2).max() / (4 * l)
        assert e <= 1e-4, e
        assert float(got[q0]) < np.sqrt(2 * l * 8 * 2.0 ** -23)


def test_noalloc_refuses_input_beyond_the_fixed_scratch():
    ctx = api.context(0)
    n, m = 6_000_000, 256
    T = torch.zeros(n, dtype=torch.float64, device="cuda")
    Q = torch.zeros(m, dtype=torch.float64, device="cuda")
    rc, _ = _noalloc(ctx, T, Q, 128, 26)
    assert rc == _lib.PST_EINVAL
    assert "fixed scratch" in ctx.L.pst_last_error(ctx.h).decode()
