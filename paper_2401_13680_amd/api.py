"""Python face of the C ABI, with the same names: mpdist_profile, profile_set,
snippets, select_length.  Inputs are float64 CUDA (ROCm) tensors; outputs are
torch tensors on the same device.  Work runs on torch's current stream.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_float, c_int32, c_void_p

import torch

from . import _lib
from ._lib import PstError, Snippet


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """A library context bound to one device and torch's current stream there,
    with a cached workspace that grows on demand."""

    def __init__(self, device: int = 0, stream=None):
        self.L = _lib.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = c_void_p()
        rc = self.L.pst_create(byref(h), device, c_void_p(stream.cuda_stream))
        if rc != 0:
            raise PstError(rc, "pst_create failed")
        self.h = h
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            self.L.pst_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def check(self, rc):
        if rc != 0:
            raise PstError(rc, self.L.pst_last_error(self.h).decode())


_default: dict = {}


def context(device: int = 0) -> Context:
    stream = torch.cuda.current_stream(device)
    key = (device, stream.cuda_stream)
    if key not in _default:
        _default[key] = Context(device, stream)
    return _default[key]


def _series(T):
    if not isinstance(T, torch.Tensor) or not T.is_cuda:
        raise TypeError("T must be a CUDA tensor (the library has no CPU path)")
    if T.dtype != torch.float64 or T.dim() != 1 or not T.is_contiguous():
        raise TypeError("T must be a contiguous 1-D float64 tensor")
    return T


def mpdist_profile(T, Q, l: int, k: int = 0, ctx: Context | None = None):
    """eq. 14: MPdist profile of Q (length m) against every length-m window of T."""
    T, Q = _series(T), _series(Q)
    ctx = ctx or context(T.device.index)
    n, m = T.numel(), Q.numel()
    nb = ctx.L.pst_workspace_bytes(n, m, l, 0)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l}")
    out = torch.empty(n - m + 1, dtype=torch.float32, device=T.device)
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_mpdist_profile(ctx.h, _ptr(T), n, _ptr(Q), m, l, k, _ptr(out),
                                        _ptr(ws), ws.numel()))
    return out


def profile_set(T, m: int, l: int, k: int = 0, ctx: Context | None = None):
    """eq. 15: all segment profiles D [n//m, n-m+1] (float32) and max(D)."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    nb = ctx.L.pst_workspace_bytes(n, m, l, 0)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l}")
    D = torch.empty((n // m, n - m + 1), dtype=torch.float32, device=T.device)
    dmax = torch.empty(1, dtype=torch.float32, device=T.device)
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_profile_set(ctx.h, _ptr(T), n, m, l, k, _ptr(D), D.stride(0), _ptr(dmax),
                                     _ptr(ws), ws.numel()))
    return D, dmax


def _records(arr, K):
    return [dict(segment=int(arr[i].segment), greedy_rank=int(arr[i].greedy_rank),
                 frac=float(arr[i].frac), area_after=float(arr[i].area_after)) for i in range(K)]


def snippets(T, m: int, l: int, K: int, k: int = 0, profiles: bool = False, owner: bool = False,
             ctx: Context | None = None):
    """Section 3.2's problem: K snippets ordered by frac (eq. 8)."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    nb = ctx.L.pst_workspace_bytes(n, m, l, K)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l} K={K}")
    Nm = n - m + 1
    prof = torch.empty((K, Nm), dtype=torch.float32, device=T.device) if profiles else None
    own = torch.empty(Nm, dtype=torch.int32, device=T.device) if owner else None
    recs = (Snippet * K)()
    dmax = c_float()
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_snippets(ctx.h, _ptr(T), n, m, l, k, K, recs, _ptr(prof), _ptr(own),
                                  byref(dmax), _ptr(ws), ws.numel()))
    return dict(records=_records(recs, K), profiles=prof, owner=own, dmax=float(dmax.value))


def snippets_blocked(T, m: int, l: int, K: int, seg_block: int = 0, k: int = 0, budget_bytes: int = 0,
                     profiles: bool = False, owner: bool = False, ctx: Context | None = None):
    """pst_snippets' result without holding the profile set whole: D is
    recomputed every greedy round in blocks of seg_block segments (or the
    largest block whose workspace fits budget_bytes)."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    if seg_block <= 0:
        seg_block = int(ctx.L.pst_snippets_blocked_max_block(n, m, l, K, budget_bytes))
        if seg_block <= 0:
            raise PstError(-1, f"no block fits {budget_bytes} bytes (n={n} m={m} l={l} K={K})")
    nb = ctx.L.pst_snippets_blocked_workspace_bytes(n, m, l, K, seg_block)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l} K={K} seg_block={seg_block}")
    Nm = n - m + 1
    prof = torch.empty((K, Nm), dtype=torch.float32, device=T.device) if profiles else None
    own = torch.empty(Nm, dtype=torch.int32, device=T.device) if owner else None
    recs = (Snippet * K)()
    dmax = c_float()
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_snippets_blocked(ctx.h, _ptr(T), n, m, l, k, K, seg_block, recs, _ptr(prof), _ptr(own),
                                          byref(dmax), _ptr(ws), ws.numel()))
    return dict(records=_records(recs, K), profiles=prof, owner=own, dmax=float(dmax.value),
                seg_block=seg_block, workspace_bytes=nb)


def snippets_multi(X, m: int, l: int, K: int, k: int = 0, owner: bool = False, ctx: Context | None = None):
    """Snippets of every coordinate of a multivariate series X (d x n, float64,
    on the GPU), the coordinates searched independently (section 3.2) in one
    batched profile launch.  Returns one pst_snippets-style result per
    coordinate."""
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64 and X.dim() == 2):
        raise TypeError("X must be a 2-D float64 CUDA tensor (d x n)")
    if X.stride(1) != 1:
        raise ValueError("X must have unit stride along the series")
    ctx = ctx or context(X.device.index)
    d, n = X.shape
    nb = ctx.L.pst_snippets_multi_workspace_bytes(d, n, m, l, K)
    if nb == 0:
        raise PstError(-1, f"invalid sizes d={d} n={n} m={m} l={l} K={K}")
    Nm = n - m + 1
    own = torch.empty((d, Nm), dtype=torch.int32, device=X.device) if owner else None
    recs = (Snippet * (d * K))()
    dmax = (c_float * d)()
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_snippets_multi(ctx.h, _ptr(X), d, X.stride(0), n, m, l, k, K, recs, _ptr(own), dmax,
                                        _ptr(ws), ws.numel()))
    return [dict(records=_records(recs[j * K:(j + 1) * K], K), owner=None if own is None else own[j],
                 dmax=float(dmax[j])) for j in range(d)]


def select_length(T, m_list, K: int, l_list=None, profiles: bool = False, owner: bool = False,
                  batched: bool = True, graph: bool = True, autotune: bool = False,
                  tune_geometry: bool = False, one_launch: bool = False, ctx: Context | None = None):
    """eq. 18: the best snippet length among m_list and its snippets.

    batched: all candidates in one persistent launch (else one after another);
    graph: capture the batched sweep as a HIP graph; autotune: tune its launch;
    tune_geometry: choose every length's tile geometry by timing first;
    one_launch: every length in one launch (else one per workgroup shape)."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_SWEEP_BATCHED, int(batched)))
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_SWEEP_GRAPH, int(graph)))
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_AUTOTUNE, int(autotune)))
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_TUNE_GEOMETRY, int(tune_geometry)))
    ctx.check(ctx.L.pst_set_option(ctx.h, _lib.PST_OPT_SWEEP_ONE_LAUNCH, int(one_launch)))
    n = T.numel()
    num = len(m_list)
    ms = (c_int32 * num)(*m_list)
    ls = (c_int32 * num)(*l_list) if l_list is not None else None
    nb = ctx.L.pst_select_length_workspace_bytes(n, ms, num, ls, K)
    if nb == 0:
        raise PstError(-1, "invalid sizes in the candidate list")
    scores = (c_double * num)()
    best = c_int32()
    recs = (Snippet * K)()
    ws = ctx.workspace(nb)
    # the profiles / owner of m_best are only known after the sweep: size for the largest Nm
    Nm_max = n - min(m_list) + 1
    prof = torch.empty((K, Nm_max), dtype=torch.float32, device=T.device) if profiles else None
    own = torch.empty(Nm_max, dtype=torch.int32, device=T.device) if owner else None
    ctx.check(ctx.L.pst_select_length(ctx.h, _ptr(T), n, ms, num, ls, K, byref(best), scores, recs,
                                       _ptr(prof), _ptr(own), _ptr(ws), ws.numel()))
    mb = int(best.value)
    Nm = n - mb + 1
    if prof is not None:
        prof = prof.view(-1)[: K * Nm].view(K, Nm)
    if own is not None:
        own = own[:Nm]
    return dict(m_best=mb, scores=list(scores), records=_records(recs, K), profiles=prof, owner=own)


def snippets_spilled(T, m: int, l: int, K: int, seg_block: int = 0, k: int = 0, budget_bytes: int = 0,
                     D_host=None, profiles: bool = False, owner: bool = False, ctx: Context | None = None):
    """snippets_blocked with the profile set kept in page-locked host memory
    (D_host, float32 (n/m, n-m+1), allocated when None) instead of recomputed
    every greedy round."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    if seg_block <= 0:
        seg_block = int(ctx.L.pst_snippets_blocked_max_block(n, m, l, K, budget_bytes))
        if seg_block <= 0:
            raise PstError(-1, f"no block fits {budget_bytes} bytes (n={n} m={m} l={l} K={K})")
    nb = ctx.L.pst_snippets_blocked_workspace_bytes(n, m, l, K, seg_block)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l} K={K} seg_block={seg_block}")
    Nm = n - m + 1
    if D_host is None:
        D_host = torch.empty((n // m, Nm), dtype=torch.float32, pin_memory=True)
    if not (D_host.dtype == torch.float32 and not D_host.is_cuda and D_host.is_contiguous()
            and tuple(D_host.shape) == (n // m, Nm)):
        raise ValueError("D_host must be a contiguous float32 host tensor of shape (n/m, n-m+1)")
    prof = torch.empty((K, Nm), dtype=torch.float32, device=T.device) if profiles else None
    own = torch.empty(Nm, dtype=torch.int32, device=T.device) if owner else None
    recs = (Snippet * K)()
    dmax = c_float()
    ws = ctx.workspace(nb)
    ctx.check(ctx.L.pst_snippets_spilled(ctx.h, _ptr(T), n, m, l, k, K, seg_block, _ptr(D_host), recs, _ptr(prof),
                                          _ptr(own), byref(dmax), _ptr(ws), ws.numel()))
    return dict(records=_records(recs, K), profiles=prof, owner=own, dmax=float(dmax.value),
                seg_block=seg_block, workspace_bytes=nb, D_host=D_host)


def select_length_blocked(T, m_list, K: int, seg_block: int, l_list=None, profiles: bool = False,
                          owner: bool = False, ctx: Context | None = None):
    """eq. 18 in bounded memory: select_length's result, every candidate's
    profile set recomputed per greedy round in blocks of seg_block segments."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    num = len(m_list)
    ms = (c_int32 * num)(*m_list)
    ls = (c_int32 * num)(*l_list) if l_list is not None else None
    nb = ctx.L.pst_select_length_blocked_workspace_bytes(n, ms, num, ls, K, seg_block)
    if nb == 0:
        raise PstError(-1, "invalid sizes in the candidate list")
    scores = (c_double * num)()
    best = c_int32()
    recs = (Snippet * K)()
    ws = ctx.workspace(nb)
    Nm_max = n - min(m_list) + 1
    prof = torch.empty((K, Nm_max), dtype=torch.float32, device=T.device) if profiles else None
    own = torch.empty(Nm_max, dtype=torch.int32, device=T.device) if owner else None
    ctx.check(ctx.L.pst_select_length_blocked(ctx.h, _ptr(T), n, ms, num, ls, K, seg_block, byref(best), scores,
                                               recs, _ptr(prof), _ptr(own), _ptr(ws), ws.numel()))
    mb = int(best.value)
    Nm = n - mb + 1
    if prof is not None:
        prof = prof.view(-1)[: K * Nm].view(K, Nm)
    if own is not None:
        own = own[:Nm]
    return dict(m_best=mb, scores=list(scores), records=_records(recs, K), profiles=prof, owner=own,
                workspace_bytes=nb)


def label_f1(owner, truth, m: int, K: int, C: int, ctx: Context | None = None):
    """Labelling score of K snippets (section 5.2's per-element F1): owner is
    the int32 owner array of snippets() (n-m+1 windows), truth the int32 true
    class of each of the n elements."""
    if not (isinstance(owner, torch.Tensor) and owner.is_cuda and owner.dtype == torch.int32):
        raise TypeError("owner must be an int32 CUDA tensor")
    if not (isinstance(truth, torch.Tensor) and truth.is_cuda and truth.dtype == torch.int32):
        raise TypeError("truth must be an int32 CUDA tensor")
    owner, truth = owner.contiguous(), truth.contiguous()
    ctx = ctx or context(truth.device.index)
    n = truth.numel()
    if owner.numel() != n - m + 1:
        raise ValueError(f"owner has {owner.numel()} windows, expected n-m+1 = {n - m + 1}")
    nb = ctx.L.pst_label_workspace_bytes(K, C)
    if nb == 0:
        raise PstError(-1, f"bad K={K} or C={C}")
    ws = ctx.workspace(nb)
    mp = (c_int32 * K)()
    prec, rec, f1 = (c_double * C)(), (c_double * C)(), (c_double * C)()
    macro = c_double()
    ctx.check(ctx.L.pst_label_f1(ctx.h, _ptr(owner), n, m, K, _ptr(truth), C, mp, prec, rec, f1,
                                 byref(macro), _ptr(ws), ws.numel()))
    return dict(map=list(mp), precision=list(prec), recall=list(rec), f1=list(f1), macro_f1=macro.value)


def torch_tensor_type():
    import torch
    return torch.Tensor


class Server:
    """Request server of the library (pst_server_*): admission by device-memory
    footprint and slots, continuous batching of the admitted requests' profile
    tiles into shared launches, results kept until polled.  Series are host
    numpy float64 arrays; each is copied on submit."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30, max_slots: int = 8):
        self.L = _lib.load()
        h = c_void_p()
        rc = self.L.pst_server_create(byref(h), device, hbm_budget_bytes, max_slots)
        if rc != 0:
            raise PstError(rc, "pst_server_create failed")
        self.h = h
        self.K = {}
        self._keep = {}   # device series of requests not yet collected

    def submit(self, x, m: int, l: int, K: int) -> int:
        """Queue series x: a host numpy array (copied now), or a CUDA float64
        tensor on the server's device, which must stay alive and unchanged
        until poll() returns the request's result."""
        t = ctypes.c_uint64()
        if isinstance(x, torch_tensor_type()):
            if not x.is_cuda or x.dtype != __import__("torch").float64 or not x.is_contiguous():
                raise ValueError("device series must be a contiguous CUDA float64 tensor")
            rc = self.L.pst_submit_device(self.h, c_void_p(x.data_ptr()), x.numel(), m, l, K, byref(t))
            self._keep[t.value] = x
        else:
            import numpy as np
            x = np.ascontiguousarray(x, dtype=np.float64)
            rc = self.L.pst_submit(self.h, c_void_p(x.ctypes.data), len(x), m, l, K, byref(t))
        if rc != 0:
            raise PstError(rc, self.L.pst_server_last_error(self.h).decode())
        self.K[t.value] = K
        return t.value

    def poll(self, ticket: int):
        """None while running; else dict(status, records, latency_ms)."""
        K = self.K[ticket]
        recs = (Snippet * K)()
        lat = c_double()
        rc = self.L.pst_poll(self.h, ticket, recs, K, byref(lat))
        if rc == _lib.PST_ENOTREADY:
            return None
        del self.K[ticket]
        self._keep.pop(ticket, None)
        return dict(status=rc, records=_records(recs, K) if rc == 0 else None, latency_ms=lat.value)

    def drain(self, timeout_ms: int = 600_000):
        rc = self.L.pst_server_drain(self.h, timeout_ms)
        if rc != 0:
            raise PstError(rc, self.L.pst_server_last_error(self.h).decode())

    ARRIVAL, SHORTEST_PREDICTED = 0, 1

    def set_policy(self, policy: int, seed: "RuntimeModel | None" = None):
        """Admission order: Server.ARRIVAL or Server.SHORTEST_PREDICTED (run
        times from a copy of `seed`, grown with every completed request)."""
        rc = self.L.pst_server_set_policy(self.h, policy, seed.h if seed is not None else None)
        if rc != 0:
            raise PstError(rc, f"bad policy {policy}")

    def stats(self):
        c, cells, a, b = ctypes.c_uint64(), c_double(), c_int32(), ctypes.c_size_t()
        self.L.pst_server_stats(self.h, byref(c), byref(cells), byref(a), byref(b))
        nb = ctypes.c_uint64()
        self.L.pst_server_batches(self.h, byref(nb))
        return dict(completed=c.value, cells=cells.value, active=a.value, bytes_in_use=b.value,
                    batches=nb.value)

    def close(self):
        if getattr(self, "h", None):
            self.L.pst_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_bytes(n: int, m: int, l: int, K: int) -> int:
    return int(_lib.load().pst_request_bytes(n, m, l, K))


class RuntimeModel:
    """Polynomial run-time model of section 4.2 (pst_model_*): observe earlier
    runs (n, m, l, ms), fit, predict.  Host-only."""

    def __init__(self, degree: int = 2):
        self.L = _lib.load()
        h = c_void_p()
        rc = self.L.pst_model_create(byref(h), degree)
        if rc != 0:
            raise PstError(rc, f"pst_model_create(degree={degree}) failed")
        self.h = h
        self.degree = degree

    def observe(self, n: int, m: int, l: int, ms: float):
        rc = self.L.pst_model_observe(self.h, n, m, l, float(ms))
        if rc != 0:
            raise PstError(rc, f"bad observation n={n} m={m} l={l} ms={ms}")

    def fit(self):
        rc = self.L.pst_model_fit(self.h)
        if rc != 0:
            raise PstError(rc, "fit failed")

    def coefficients(self):
        num = c_int32()
        rc = self.L.pst_model_coefficients(self.h, None, 0, byref(num))
        if rc != 0:
            raise PstError(rc, "model not fitted")
        out = (c_double * num.value)()
        self.L.pst_model_coefficients(self.h, out, num.value, byref(num))
        return list(out)

    def predict(self, n: int, m: int, l: int) -> float:
        out = c_double()
        rc = self.L.pst_model_predict(self.h, n, m, l, byref(out))
        if rc != 0:
            raise PstError(rc, f"cannot predict n={n} m={m} l={l}")
        return out.value

    def close(self):
        if getattr(self, "h", None):
            self.L.pst_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition_kk(costs, parts: int):
    """Karmarkar-Karp k-way partition (pst_partition_kk): (part of each item, load of each part)."""
    L = _lib.load()
    cnt = len(costs)
    c = (c_double * max(cnt, 1))(*[float(x) for x in costs])
    po = (c_int32 * max(cnt, 1))()
    lo = (c_double * parts)()
    rc = L.pst_partition_kk(c, cnt, parts, po, lo)
    if rc != 0:
        raise PstError(rc, "pst_partition_kk failed")
    return list(po)[:cnt], list(lo)


def partition_lengths(model: RuntimeModel, n: int, m_list, parts: int, l_list=None):
    """Candidate lengths spread over `parts` workers by predicted run time."""
    L = _lib.load()
    k = len(m_list)
    ms = (c_int32 * k)(*m_list)
    ls = (c_int32 * k)(*l_list) if l_list is not None else None
    po = (c_int32 * k)()
    lo = (c_double * parts)()
    rc = L.pst_partition_lengths(model.h, n, ms, ls, k, parts, po, lo)
    if rc != 0:
        raise PstError(rc, "pst_partition_lengths failed")
    return list(po), list(lo)


# ---------------------------------------------------------------- tile geometry
def decode_geometry(code: int) -> dict:
    """The profile kernel's tile geometry from its code (include/pst.h)."""
    return dict(threads=((code >> 24) & 0xF) * 256, diagonals_per_thread=(code >> 16) & 0xFF,
                rows_per_chunk=(code >> 8) & 0xFF, selection_threads=((code >> 4) & 0xF) * 256,
                subtile_windows=(code & 0xF) * 992)


def geometry_candidates(w: int) -> list:
    L = _lib.load()
    n = L.pst_geometry_candidates(w, None, 0)
    buf = (c_int32 * max(n, 1))()
    L.pst_geometry_candidates(w, buf, n)
    return list(buf)[:n]


def geometry(w: int) -> int:
    return int(_lib.load().pst_geometry(w))


def set_geometry(w: int, code: int):
    rc = _lib.load().pst_set_geometry(w, code)
    if rc != 0:
        raise PstError(rc, f"geometry {code:#x} is not a candidate for w={w}")


def tune_geometry(T, m: int, l: int, ctx: Context | None = None):
    """Time every tile geometry for w = m-l+1 on T's segment profiles and
    install the fastest (process-wide); returns (code, ms)."""
    T = _series(T)
    ctx = ctx or context(T.device.index)
    n = T.numel()
    nb = ctx.L.pst_workspace_bytes(n, m, l, 1)
    if nb == 0:
        raise PstError(-1, f"invalid sizes n={n} m={m} l={l}")
    ws = ctx.workspace(nb)
    code, ms = c_int32(), c_float()
    ctx.check(ctx.L.pst_tune_geometry(ctx.h, _ptr(T), n, m, l, byref(code), byref(ms), _ptr(ws), ws.numel()))
    return code.value, ms.value
