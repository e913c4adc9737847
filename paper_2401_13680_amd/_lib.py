"""ctypes binding of libpst.so (include/pst.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Torch provides device memory and the current stream.  There is no
CPU fallback; a missing library or a CPU tensor is an error.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpst.so")
# a build whose profile kernel counts its phases (analysis only; bench.py --workload probe)
PROBE_LIB_PATH = os.path.join(HERE, "libpst_probe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pst.h")

PST_OK, PST_EINVAL, PST_ENOMEM, PST_EDEVICE, PST_ENOTREADY, PST_ECANCELED = 0, -1, -2, -3, -4, -5
PST_OPT_SWEEP_GRAPH, PST_OPT_AUTOTUNE, PST_OPT_PROFILE_GRID, PST_OPT_DYNAMIC_TILES, \
    PST_OPT_SWEEP_BATCHED, PST_OPT_ANCHOR_EVERY, PST_OPT_TUNE_GEOMETRY, PST_OPT_SWEEP_ONE_LAUNCH = \
    1, 2, 3, 4, 5, 6, 7, 8
STATUS_NAMES = {0: "PST_OK", -1: "PST_EINVAL", -2: "PST_ENOMEM", -3: "PST_EDEVICE",
                -4: "PST_ENOTREADY", -5: "PST_ECANCELED"}


class Snippet(ctypes.Structure):
    _fields_ = [("segment", c_int32), ("greedy_rank", c_int32),
                ("frac", c_double), ("area_after", c_double)]


class PstError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def header_functions():
    """Names of the functions that include/pst.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pst_[a-z_]+)\s*\(", txt)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2401_13680_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "pst_version": (c_char_p, []),
        "pst_create": (c_int, [POINTER(P), c_int, P]),
        "pst_destroy": (None, [P]),
        "pst_last_error": (c_char_p, [P]),
        "pst_workspace_bytes": (c_size_t, [c_int64, c_int32, c_int32, c_int32]),
        "pst_select_length_workspace_bytes": (c_size_t, [c_int64, POINTER(c_int32), c_int32,
                                                         POINTER(c_int32), c_int32]),
        "pst_mpdist_profile": (c_int, [P, P, c_int64, P, c_int32, c_int32, c_int32, P, P, c_size_t]),
        "pst_mpdist_profile_noalloc": (c_int, [P, P, c_int64, P, c_int32, c_int32, c_int32, P]),
        "pst_profile_set": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, P, c_int64, P, P,
                                    c_size_t]),
        "pst_snippets": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, c_int32,
                                 POINTER(Snippet), P, P, POINTER(c_float), P, c_size_t]),
        "pst_select_length": (c_int, [P, P, c_int64, POINTER(c_int32), c_int32, POINTER(c_int32),
                                      c_int32, POINTER(c_int32), POINTER(c_double),
                                      POINTER(Snippet), P, P, P, c_size_t]),
        "pst_snippets_blocked_workspace_bytes": (c_size_t, [c_int64, c_int32, c_int32, c_int32, c_int32]),
        "pst_snippets_blocked_max_block": (c_int32, [c_int64, c_int32, c_int32, c_int32, c_size_t]),
        "pst_snippets_blocked": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, c_int32, c_int32,
                                         POINTER(Snippet), P, P, POINTER(c_float), P, c_size_t]),
        "pst_snippets_spilled": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, c_int32, c_int32, P,
                                         POINTER(Snippet), P, P, POINTER(c_float), P, c_size_t]),
        "pst_select_length_blocked_workspace_bytes": (c_size_t, [c_int64, POINTER(c_int32), c_int32,
                                                                 POINTER(c_int32), c_int32, c_int32]),
        "pst_select_length_blocked": (c_int, [P, P, c_int64, POINTER(c_int32), c_int32, POINTER(c_int32), c_int32,
                                              c_int32, POINTER(c_int32), POINTER(c_double), POINTER(Snippet), P, P,
                                              P, c_size_t]),
        "pst_snippets_multi_workspace_bytes": (c_size_t, [c_int32, c_int64, c_int32, c_int32, c_int32]),
        "pst_snippets_multi": (c_int, [P, P, c_int32, c_int64, c_int64, c_int32, c_int32, c_int32, c_int32,
                                       POINTER(Snippet), P, POINTER(c_float), P, c_size_t]),
        "pst_model_create": (c_int, [POINTER(P), c_int32]),
        "pst_model_destroy": (None, [P]),
        "pst_model_observe": (c_int, [P, c_int64, c_int32, c_int32, c_double]),
        "pst_model_fit": (c_int, [P]),
        "pst_model_coefficients": (c_int, [P, POINTER(c_double), c_int32, POINTER(c_int32)]),
        "pst_model_predict": (c_int, [P, c_int64, c_int32, c_int32, POINTER(c_double)]),
        "pst_partition_kk": (c_int, [POINTER(c_double), c_int32, c_int32, POINTER(c_int32), POINTER(c_double)]),
        "pst_partition_lengths": (c_int, [P, c_int64, POINTER(c_int32), POINTER(c_int32), c_int32, c_int32,
                                          POINTER(c_int32), POINTER(c_double)]),
        "pst_set_timing": (c_int, [P, c_int]),
        "pst_set_option": (c_int, [P, c_int, c_int64]),
        "pst_geometry_candidates": (c_int, [c_int32, POINTER(c_int32), c_int32]),
        "pst_geometry": (c_int32, [c_int32]),
        "pst_set_geometry": (c_int, [c_int32, c_int32]),
        "pst_tune_geometry": (c_int, [P, P, c_int64, c_int32, c_int32, POINTER(c_int32), POINTER(c_float), P,
                                      c_size_t]),
        "pst_server_create": (c_int, [POINTER(P), c_int, c_size_t, c_int32]),
        "pst_server_destroy": (None, [P]),
        "pst_server_last_error": (c_char_p, [P]),
        "pst_request_bytes": (c_size_t, [c_int64, c_int32, c_int32, c_int32]),
        "pst_pool_size_class": (c_int, [c_size_t, POINTER(c_size_t)]),
        "pst_server_batches": (c_int, [P, POINTER(ctypes.c_uint64)]),
        "pst_submit": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, POINTER(ctypes.c_uint64)]),
        "pst_submit_device": (c_int, [P, P, c_int64, c_int32, c_int32, c_int32, POINTER(ctypes.c_uint64)]),
        "pst_poll": (c_int, [P, ctypes.c_uint64, POINTER(Snippet), c_int32, POINTER(c_double)]),
        "pst_server_drain": (c_int, [P, c_int32]),
        "pst_server_stats": (c_int, [P, POINTER(ctypes.c_uint64), POINTER(c_double), POINTER(c_int32),
                                     POINTER(c_size_t)]),
        "pst_admission_simulate": (c_int, [c_size_t, c_int32, c_int32, POINTER(c_size_t),
                                           POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
        "pst_admission_simulate_ordered": (c_int, [c_size_t, c_int32, c_int32, POINTER(c_size_t),
                                                   POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                                   POINTER(c_double)]),
        "pst_server_set_policy": (c_int, [P, c_int32, P]),
        "pst_last_profile_ms": (c_int, [P, POINTER(c_float)]),
        "pst_label_workspace_bytes": (c_size_t, [c_int32, c_int32]),
        "pst_label_f1": (c_int, [P, P, c_int64, c_int32, c_int32, P, c_int32, POINTER(c_int32),
                                 POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                 POINTER(c_double), P, c_size_t]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
