"""Workspace-size functions of the C ABI (host only, no GPU): zero for invalid
sizes, growth with the problem, the bounded-memory block search against its
own size function, and the multivariate and sweep sizes against the
single-problem ones."""
import ctypes

from paper_2401_13680_amd import _lib

L = _lib.load()


def _arr(vals):
    return (ctypes.c_int32 * len(vals))(*vals)


def test_invalid_sizes_give_zero():
    assert L.pst_workspace_bytes(100, 200, 50, 1) == 0          # n < m
    assert L.pst_workspace_bytes(1000, 100, 101, 1) == 0        # l > m
    assert L.pst_workspace_bytes(1000, 100, 50, 11) == 0        # K > n/m
    assert L.pst_snippets_blocked_workspace_bytes(1000, 100, 50, 3, 0) == 0
    assert L.pst_snippets_blocked_workspace_bytes(1000, 100, 50, 3, 11) == 0
    assert L.pst_snippets_multi_workspace_bytes(0, 1000, 100, 50, 3) == 0
    assert L.pst_snippets_multi_workspace_bytes(17, 1000, 100, 50, 3) == 0
    assert L.pst_select_length_blocked_workspace_bytes(1000, _arr([100, 2000]), 2, None, 3, 4) == 0
    assert L.pst_request_bytes(100, 200, 50, 1) == 0


def test_sizes_grow_with_the_problem():
    a = L.pst_workspace_bytes(100_000, 256, 128, 4)
    b = L.pst_workspace_bytes(200_000, 256, 128, 4)
    assert 0 < a < b
    # a server request holds the series and the workspace without the profile
    # scratch (batches share one scratch per batch stream): at least the profile
    # set and the series, less than the standalone workspace
    r = L.pst_request_bytes(100_000, 256, 128, 4)
    nseg, Nm = 100_000 // 256, 100_000 - 256 + 1
    assert 4 * nseg * Nm + 8 * 100_000 <= r < a + 8 * 100_000


def test_pool_size_classes():
    import ctypes
    got = ctypes.c_size_t()
    prev = 0
    for b in (1, 1 << 20, (1 << 20) + 1, 3 << 20, 1 << 30, 123456789):
        assert L.pst_pool_size_class(b, ctypes.byref(got)) == 0
        c = got.value
        assert c >= b and c >= 1 << 20
        assert c <= max(1 << 20, int(b * 1.25) + 1)     # classes 25 % apart
    # the same class for every size inside it
    L.pst_pool_size_class(5 << 20, ctypes.byref(got))
    c = got.value
    L.pst_pool_size_class(c, ctypes.byref(got))
    assert got.value == c


def test_blocked_block_search():
    n, m, l, K = 1_000_000, 256, 128, 4
    nseg = n // m
    full = L.pst_snippets_blocked_workspace_bytes(n, m, l, K, nseg)
    one = L.pst_snippets_blocked_workspace_bytes(n, m, l, K, 1)
    assert 0 < one < full
    for budget in (one - 1, one, 1 << 30, 4 << 30, full, full * 2):
        b = L.pst_snippets_blocked_max_block(n, m, l, K, budget)
        if budget < one:
            assert b == 0
            continue
        assert 1 <= b <= nseg
        assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, b) <= budget
        if b < nseg:
            assert L.pst_snippets_blocked_workspace_bytes(n, m, l, K, b + 1) > budget


def test_multi_and_sweep_sizes():
    n, m, l, K = 100_000, 256, 128, 4
    one = L.pst_workspace_bytes(n, m, l, K)
    four = L.pst_snippets_multi_workspace_bytes(4, n, m, l, K)
    assert four > 0
    # four coordinates share one profile scratch: less than four single workspaces
    assert four < 4 * one
    ms = [64, 128, 256]
    blocked = L.pst_select_length_blocked_workspace_bytes(n, _arr(ms), 3, None, K, 50)
    batched = L.pst_select_length_workspace_bytes(n, _arr(ms), 3, None, K)
    assert 0 < blocked < batched
