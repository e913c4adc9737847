"""CPU oracle for the scheduling of section 4.2: polynomial regression of run
time on earlier runs, and the Karmarkar-Karp partition of candidate lengths
over workers.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the product path never
imports it and it shares no code with the library.

The paper names the two techniques without their details; the readings (also
in the design notes) are:

  * the model is a polynomial of total degree D in three scaled sizes of a
    run: u = floor(n/m)/1e3 segments, w = (m-l+1)/1e2 window width,
    v = (n-l+1)/1e5 subsequences, whose product is proportional to the
    distance-matrix cell count; monomials in graded order (total degree
    t = 0..D, then the power of u from t down, then the power of w from what
    is left down);
  * it minimises the relative squared error of the run times, with a ridge of
    1e-10 times the mean squared column norm of the weighted design matrix;
  * the partition is the k-way largest differencing method: items start as
    k-tuples (cost, 0, .., 0); the two tuples of largest spread (ties to the
    older one, items older than merges and in input order) are merged slot by
    slot, largest slot of one with smallest of the other, the merged slots
    re-sorted largest first (stably), until one tuple is left.
"""
from __future__ import annotations

import heapq

import numpy as np


def scaled_sizes(n: int, m: int, l: int):
    return (n // m) / 1e3, (m - l + 1) / 1e2, (n - l + 1) / 1e5


def monomial_exponents(D: int):
    out = []
    for t in range(D + 1):
        for a in range(t, -1, -1):
            for b in range(t - a, -1, -1):
                out.append((a, b, t - a - b))
    return out


def design_row(D: int, n: int, m: int, l: int) -> np.ndarray:
    u, w, v = scaled_sizes(n, m, l)
    return np.array([u ** a * w ** b * v ** c for a, b, c in monomial_exponents(D)])


def fit(D: int, runs) -> np.ndarray:
    """Coefficients from runs [(n, m, l, ms), ...]."""
    A = np.array([design_row(D, n, m, l) / ms for n, m, l, ms in runs])
    y = np.ones(len(runs))
    P = A.shape[1]
    lam = np.sqrt(1e-10 * np.sum(A * A) / P)
    Aa = np.vstack([A, lam * np.eye(P)])
    ya = np.concatenate([y, np.zeros(P)])
    coef, *_ = np.linalg.lstsq(Aa, ya, rcond=None)
    return coef


def predict(D: int, coef: np.ndarray, n: int, m: int, l: int) -> float:
    return float(design_row(D, n, m, l) @ coef)


def kk_partition(costs, k: int):
    """(part of each item, load of each part), parts numbered by load, largest first."""
    tuples = {}
    heap = []
    for i, c in enumerate(costs):
        tuples[i] = ([float(c)] + [0.0] * (k - 1), [[i]] + [[] for _ in range(k - 1)])
        heapq.heappush(heap, (-(tuples[i][0][0] - tuples[i][0][-1]), i))
    nxt = len(costs)
    while len(heap) > 1:
        _, a = heapq.heappop(heap)
        _, b = heapq.heappop(heap)
        sa, ia = tuples.pop(a)
        sb, ib = tuples.pop(b)
        s = [sa[j] + sb[k - 1 - j] for j in range(k)]
        it = [ia[j] + ib[k - 1 - j] for j in range(k)]
        order = sorted(range(k), key=lambda j: -s[j])     # sorted() is stable
        tuples[nxt] = ([s[j] for j in order], [it[j] for j in order])
        heapq.heappush(heap, (-(tuples[nxt][0][0] - tuples[nxt][0][-1]), nxt))
        nxt += 1
    part = [0] * len(costs)
    if not heap:
        return part, [0.0] * k
    s, it = tuples[heap[0][1]]
    for j in range(k):
        for i in it[j]:
            part[i] = j
    return part, list(s)
