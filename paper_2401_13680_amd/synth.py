"""Seeded synthetic series for tests, benchmarks and serving replays.

The paper evaluates on public datasets (TSSB, Solar Power, PAMAP; section 5.1.1)
that are not available here.  These generators stand in for them: regime-switching
series whose regimes are periodic shapes of random period, amplitude and length,
plus Gaussian noise, with per-point ground-truth regime labels kept alongside.

This module holds no arithmetic of the method (no z-normalisation, no distances):
it only draws inputs.  Both the CPU checker and the GPU path consume its arrays.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SHAPES5 = ("sine", "square", "sawtooth", "chirp", "pulse")
SHAPES6 = SHAPES5 + ("walk",)


def _shape(kind: str, t: np.ndarray, period: float, amp: float, rng, level: float):
    """One regime of length len(t); t is local time 0..L-1."""
    L = len(t)
    if kind == "sine":
        return amp * np.sin(2.0 * np.pi * t / period)
    if kind == "square":
        s = np.sin(2.0 * np.pi * t / period)
        return amp * np.where(s >= 0.0, 1.0, -1.0)
    if kind == "sawtooth":
        u = t / period
        return amp * (2.0 * (u - np.floor(u)) - 1.0)
    if kind == "chirp":
        p0, p1 = period, period / 4.0
        ph = t / p0 + (p0 / p1 - 1.0) * t * t / (2.0 * p0 * max(L, 1))
        return amp * np.sin(2.0 * np.pi * ph)
    if kind == "pulse":
        u = np.mod(t, period) / period
        return amp * np.exp(-3.0 * u) * np.sin(6.0 * np.pi * u)
    if kind == "walk":
        return level + np.cumsum(rng.normal(0.0, 0.1, size=L))
    raise ValueError(kind)


@dataclass
class Series:
    x: np.ndarray          # float64[n]
    labels: np.ndarray     # int32[n], regime shape id per point
    shapes: tuple


def regime_series(n: int, seed: int, shapes=SHAPES5, len_range=(2000, 8000),
                  amp_range=(0.5, 2.0), period_range=(20, 200), noise=0.1) -> Series:
    """Regime-switching series: consecutive regimes have different shapes."""
    rng = np.random.default_rng(seed)
    x = np.empty(n, dtype=np.float64)
    lab = np.empty(n, dtype=np.int32)
    pos, prev, level = 0, -1, 0.0
    while pos < n:
        L = int(rng.integers(len_range[0], len_range[1] + 1))
        L = min(L, n - pos)
        k = int(rng.integers(0, len(shapes)))
        if k == prev:
            k = (k + 1 + int(rng.integers(0, len(shapes) - 1))) % len(shapes)
        period = float(rng.integers(period_range[0], period_range[1] + 1))
        amp = float(rng.uniform(amp_range[0], amp_range[1]))
        seg = _shape(shapes[k], np.arange(L, dtype=np.float64), period, amp, rng, level)
        x[pos:pos + L] = seg
        lab[pos:pos + L] = k
        level = float(seg[-1]) if shapes[k] == "walk" else 0.0
        pos += L
        prev = k
    x += rng.normal(0.0, noise, size=n)
    return Series(x, lab, tuple(shapes))


@dataclass
class MultiSeries:
    x: np.ndarray          # float64[d, n], coordinate j in row j
    labels: np.ndarray     # int32[n], regime class per point (shared by all coordinates)


def multivariate_series(n: int, d: int, seed: int, shapes=SHAPES5, len_range=(2000, 8000),
                        amp_range=(0.5, 2.0), period_range=(20, 200), noise=0.1) -> MultiSeries:
    """d coordinates switching regime at the same points (one activity seen by
    d sensors): a regime of class c is drawn in coordinate j with the shape
    perm_j[c], its own period and amplitude, plus N(0, noise) per coordinate.
    Consecutive regimes have different classes."""
    rng = np.random.default_rng(seed)
    C = len(shapes)
    perms = [rng.permutation(C) for _ in range(d)]
    x = np.empty((d, n), dtype=np.float64)
    lab = np.empty(n, dtype=np.int32)
    pos, prev = 0, -1
    level = np.zeros(d)
    while pos < n:
        L = min(int(rng.integers(len_range[0], len_range[1] + 1)), n - pos)
        c = int(rng.integers(0, C))
        if c == prev:
            c = (c + 1 + int(rng.integers(0, C - 1))) % C
        t = np.arange(L, dtype=np.float64)
        for j in range(d):
            kind = shapes[perms[j][c]]
            period = float(rng.integers(period_range[0], period_range[1] + 1))
            amp = float(rng.uniform(amp_range[0], amp_range[1]))
            seg = _shape(kind, t, period, amp, rng, level[j])
            x[j, pos:pos + L] = seg
            level[j] = float(seg[-1]) if kind == "walk" else 0.0
        lab[pos:pos + L] = c
        pos += L
        prev = c
    x += rng.normal(0.0, noise, size=(d, n))
    return MultiSeries(x, lab)


def four_regimes(seed: int = 1) -> Series:
    """n=2000: sine P=50, square P=40, sawtooth P=60, random walk sigma 0.1,
    500 points each, plus N(0, 0.05) noise."""
    rng = np.random.default_rng(seed)
    t = np.arange(500, dtype=np.float64)
    parts = [
        _shape("sine", t, 50.0, 1.0, rng, 0.0),
        _shape("square", t, 40.0, 1.0, rng, 0.0),
        _shape("sawtooth", t, 60.0, 1.0, rng, 0.0),
        _shape("walk", t, 0.0, 1.0, rng, 0.0),
    ]
    x = np.concatenate(parts) + rng.normal(0.0, 0.05, size=2000)
    lab = np.repeat(np.arange(4, dtype=np.int32), 500)
    return Series(x, lab, ("sine", "square", "sawtooth", "walk"))


def long_walk(n: int = 1_000_000, seed: int = 4, n_planted: int = 10,
              planted_len: int = 10_000, amp: float = 10.0) -> Series:
    """Random-walk base (cumulative N(0,1)) with planted periodic regimes,
    noise sigma 0.05, rounded to float32 and widened back exactly."""
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(0.0, 1.0, size=n))
    lab = np.zeros(n, dtype=np.int32)
    kinds = ("sine", "square", "sawtooth")
    for r in range(n_planted):
        start = 50_000 + 100_000 * r
        if start + planted_len > n:
            break
        period = float(rng.integers(64, 257))
        seg = _shape(kinds[r % 3], np.arange(planted_len, dtype=np.float64), period, amp, rng, 0.0)
        x[start:start + planted_len] += seg
        lab[start:start + planted_len] = 1 + (r % 3)
    x += rng.normal(0.0, 0.05, size=n)
    x = x.astype(np.float32).astype(np.float64)
    return Series(x, lab, ("walk",) + kinds)


def planted_motifs(m: int, n_motifs: int, copies, seed: int, noise: float = 0.0):
    """Series made of segment-aligned copies of distinct random motifs.

    ``copies`` is a list (one per motif) of copy counts.  Returns (x, order)
    where order[s] is the motif id of segment s.  Exact copies of one motif
    are bit-identical segments.
    """
    rng = np.random.default_rng(seed)
    motifs = [np.cumsum(rng.normal(0.0, 1.0, size=m)) + 3.0 * np.sin(
        2.0 * np.pi * np.arange(m) / rng.integers(8, max(9, m // 2)))
        for _ in range(n_motifs)]
    order = np.concatenate([np.full(c, i) for i, c in enumerate(copies)])
    rng.shuffle(order)
    x = np.concatenate([motifs[i] for i in order])
    if noise:
        x = x + rng.normal(0.0, noise, size=len(x))
    return x.astype(np.float64), order


def random_tiny(n: int, seed: int) -> np.ndarray:
    """A short random walk with a sine, for brute-force comparisons."""
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64)
    return np.cumsum(rng.normal(0, 1, n)) * 0.3 + np.sin(2 * np.pi * t / rng.integers(5, 30))


# ---------------------------------------------------------------- workloads
# Named workloads with the sizes the benchmarks and parity tests use.
WORKLOADS = {
    "four_regimes_n2000": dict(n=2000, m=100, l=50, K=3),
    "regimes5_n100000": dict(n=100_000, m=256, l=128, K=4),
    "regimes6_n250000_sweep": dict(n=250_000, m_list=list(range(64, 513, 32)), K=6),
    "walk_n1000000": dict(n=1_000_000, m=512, l=256, K=4),
    "multi4_n100000": dict(n=100_000, d=4, m=256, l=128, K=4),
}


def default_k(m: int) -> int:
    """ceil(0.05 * 2m) in integer arithmetic: the paper's typical k."""
    return (m + 9) // 10


def workload_series(name: str) -> np.ndarray:
    if name == "four_regimes_n2000":
        return four_regimes(1).x
    if name == "regimes5_n100000":
        return regime_series(100_000, 2, SHAPES5).x
    if name == "regimes6_n250000_sweep":
        return regime_series(250_000, 3, SHAPES6).x
    if name == "walk_n1000000":
        return long_walk(1_000_000, 4).x
    if name == "multi4_n100000":
        return multivariate_series(100_000, 4, 6).x
    raise KeyError(name)


@dataclass
class Request:
    arrival_s: float
    x: np.ndarray
    m: int
    l: int
    K: int


def poisson_requests(num: int = 200, rate: float = 20.0, seed: int = 5,
                     n_range=(10_000, 500_000), m_choices=(64, 128, 256, 512, 1024)):
    """Poisson arrivals of independent regime-switching series, n log-uniform."""
    master = np.random.default_rng(seed)
    children = np.random.SeedSequence(seed).spawn(num)
    t, out = 0.0, []
    for i in range(num):
        t += float(master.exponential(1.0 / rate))
        n = int(round(math.exp(master.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        m = int(master.choice(m_choices))
        K = int(master.integers(3, 6))
        cseed = int(children[i].generate_state(1)[0])
        x = regime_series(n, cseed, SHAPES5).x
        out.append(Request(t, x, m, m // 2, K))
    return out
