"""Host-side checks of the C ABI: the library loads, exports every function
that include/pst.h declares, sizes its workspace, and rejects bad sizes.
No compute call is made here (no GPU needed)."""
import ctypes

import pytest

from paper_2401_13680_amd import _lib


def test_exports_every_declared_function():
    L = _lib.load()
    names = _lib.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_version():
    assert b"gfx950" in _lib.load().pst_version()


def test_workspace_bytes():
    L = _lib.load()
    small = L.pst_workspace_bytes(2000, 100, 50, 3)
    big = L.pst_workspace_bytes(100_000, 256, 128, 4)
    assert 0 < small < big
    # the profile set alone is nseg * Nm floats
    assert big >= 4 * (100_000 // 256) * (100_000 - 256 + 1)
    ms = (ctypes.c_int32 * 3)(64, 128, 256)
    sweep = L.pst_select_length_workspace_bytes(100_000, ms, 3, None, 4)
    assert sweep >= L.pst_workspace_bytes(100_000, 64, 32, 4)


@pytest.mark.parametrize("n,m,l,K", [
    (100, 200, 50, 1),     # m > n
    (1000, 100, 1, 1),     # l < 2
    (1000, 100, 101, 1),   # l > m
    (1000, 100, 50, 11),   # K > n/m
    (1000, 100, 50, -1),   # K < 0
    (10_000, 3000, 20, 1), # w too large
])
def test_workspace_rejects_invalid(n, m, l, K):
    assert _lib.load().pst_workspace_bytes(n, m, l, K) == 0


def test_null_context_and_no_device():
    import torch
    L = _lib.load()
    assert L.pst_last_error(None) == b"null context"
    if not torch.cuda.is_available():
        h = ctypes.c_void_p()
        assert L.pst_create(ctypes.byref(h), 0, None) == _lib.PST_EDEVICE
        assert not h.value
