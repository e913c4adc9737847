"""Host logic of the profile kernel's tile geometries (no GPU): every
candidate decodes to a workgroup the kernels exist for, the built-in choice
is a candidate, an override must be a candidate and can be undone, and
workspace sizes already cover every candidate (they do not change when one
is installed)."""
import pytest

from paper_2401_13680_amd import _lib, api

L = _lib.load()


@pytest.mark.parametrize("w", [1, 2, 33, 65, 129, 180, 181, 257, 300, 513, 700, 1025])
def test_candidates_and_builtin(w):
    codes = api.geometry_candidates(w)
    assert codes, w
    kernels = {(256, 5, 8), (256, 6, 8), (512, 5, 8), (512, 5, 4), (512, 6, 4)}
    for c in codes:
        g = api.decode_geometry(c)
        assert (g["threads"], g["diagonals_per_thread"], g["rows_per_chunk"]) in kernels, hex(c)
        assert g["selection_threads"] in (256, 512) and g["selection_threads"] <= g["threads"]
        assert g["subtile_windows"] in (992, 1984)
    assert api.geometry(w) in codes
    assert len(set(codes)) == len(codes)


def test_override_must_be_a_candidate_and_can_be_undone():
    w = 129
    builtin = api.geometry(w)
    others = [c for c in api.geometry_candidates(w) if c != builtin]
    assert others
    assert L.pst_set_geometry(w, 0x7123456) != 0          # not a candidate
    assert api.geometry(w) == builtin
    assert L.pst_set_geometry(w, others[0]) == 0
    try:
        assert api.geometry(w) == others[0]
    finally:
        assert L.pst_set_geometry(w, 0) == 0
    assert api.geometry(w) == builtin
    assert L.pst_set_geometry(0, others[0]) != 0          # w out of range
    assert L.pst_set_geometry(1026, others[0]) != 0


@pytest.mark.parametrize("n,m", [(20_000, 64), (100_000, 256), (50_000, 1024)])
def test_workspace_covers_every_candidate(n, m):
    l = m // 2
    w = m - l + 1
    base = L.pst_workspace_bytes(n, m, l, 3)
    try:
        for c in api.geometry_candidates(w):
            assert L.pst_set_geometry(w, c) == 0
            assert L.pst_workspace_bytes(n, m, l, 3) == base, hex(c)
    finally:
        L.pst_set_geometry(w, 0)
