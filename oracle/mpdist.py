"""FP64 CPU oracle for MPdist profiles, snippets and the snippet-length criterion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
It shares no code with the GPU library and never reads any of its outputs.

Every function follows the paper's definitions in the paper's order, in plain
numpy float64 (0-based indices; the paper is 1-based):

  eq. 3-4    subsequences and non-overlapping segments
  eq. 9      ED_matr: z-normalised Euclidean distances between the segment's
             length-l subsequences and all length-l subsequences of T,
             evaluated through the dot-product form of ref. [7]
  eq. 10     allP_BA: column minima of ED_matr
  eq. 11     allP_AB: row minima over a sliding window of w = m-l+1 columns
  eq. 12-13  P_ABBA concatenation; MPdist = its k-th smallest element
             (the largest one when P_ABBA has no more than k elements)
  eq. 14-15  MPdist profile MPD(Q, T) and the profile set D
  eq. 16-17  representativeness curve M and ProfileArea
  eq. 6-8    neighbours, frac and the ordering of snippets
  eq. 18     the snippet-length criterion
  eq. 1-2    a multivariate series: section 3.2 searches each coordinate on
             its own, so the multivariate result is the list of the
             coordinates' results

Readings taken where the text is garbled or silent (each is also listed in the
design notes): sliding window width w = m-l+1 in eq. 11; element min(k, 2w) in
eq. 13; population sigma, and an all-zero z-vector for a constant window; the
curve and the area run over all n-m+1 windows; greedy selection of the segment
that lowers the area most, ties to the lowest index; neighbours are counted
among the K chosen snippets, ties to the earliest pick; eq. 18's denominator is
the maximum over every entry of D; the tail after the last whole segment is
not a segment.
"""
from __future__ import annotations

import numpy as np

sliding = np.lib.stride_tricks.sliding_window_view


def default_k(m: int) -> int:
    """Typical k of eq. 13: 5 % of 2m, rounded up, in integer arithmetic."""
    return (m + 9) // 10


def const_threshold(x: np.ndarray) -> float:
    """A window whose population sigma is at or below this is treated as constant."""
    return 1e-6 * max(1.0, float(np.max(np.abs(x)))) if len(x) else 1e-6


def window_stats(x: np.ndarray, l: int):
    """Two-pass mean and population standard deviation of every length-l subsequence."""
    W = sliding(np.asarray(x, dtype=np.float64), l)
    mu = W.mean(axis=1)
    sig = np.sqrt(((W - mu[:, None]) ** 2).mean(axis=1))
    const = sig <= const_threshold(x)
    return mu, sig, const


def znorm_matrix(x: np.ndarray, l: int) -> np.ndarray:
    """Rows are the z-normalised length-l subsequences T_{j,l}; a constant one is all zero."""
    W = sliding(np.asarray(x, dtype=np.float64), l)
    mu, sig, const = window_stats(x, l)
    Z = (W - mu[:, None]) / np.where(const, 1.0, sig)[:, None]
    Z[const] = 0.0
    return Z


def ed_matr(Zq: np.ndarray, Zt: np.ndarray) -> np.ndarray:
    """eq. 9: ED_norm between every row of Zq and every row of Zt.

    Uses ||a-b||^2 = ||a||^2 + ||b||^2 - 2<a,b> on z-normalised rows (the
    dot-product technique of ref. [7]); negative rounding residue is clamped.
    """
    na = np.einsum("ij,ij->i", Zq, Zq)
    nb = np.einsum("ij,ij->i", Zt, Zt)
    d2 = na[:, None] + nb[None, :] - 2.0 * (Zq @ Zt.T)
    return np.sqrt(np.maximum(d2, 0.0))


def mpd_from_ed(E: np.ndarray, k: int) -> np.ndarray:
    """eqs. 10-13 applied to ED_matr E of shape (w, n-l+1); returns n-m+1 values."""
    w = E.shape[0]
    allP_BA = E.min(axis=0)                                  # eq. 10
    allP_AB = sliding(E, w, axis=1).min(axis=2)              # eq. 11, shape (w, n-m+1)
    Nm = allP_AB.shape[1]
    P_ABBA = np.concatenate([allP_AB.T, sliding(allP_BA, w)[:Nm]], axis=1)   # eq. 12
    SortedP = np.sort(P_ABBA, axis=1)
    idx = min(k, 2 * w) - 1                                  # eq. 13 (1-based k)
    return SortedP[:, idx]


def mpd(q: np.ndarray, x: np.ndarray, l: int, k: int | None = None) -> np.ndarray:
    """eq. 14: MPdist profile of Q (length m) against every length-m window of T."""
    q = np.asarray(q, dtype=np.float64)
    m = len(q)
    k = default_k(m) if k is None else k
    Zq = znorm_matrix(q, l)
    Zt = znorm_matrix(x, l)
    return mpd_from_ed(ed_matr(Zq, Zt), k)


def mpdist(a: np.ndarray, b: np.ndarray, l: int, k: int | None = None) -> float:
    """MPdist between two sequences of equal length m (eq. 13)."""
    assert len(a) == len(b)
    return float(mpd(a, b, l, k)[0])


def mpdist_samples(x: np.ndarray, m: int, l: int, k: int, pairs) -> np.ndarray:
    """D_s(j) for a list of (s, j) pairs, each computed on its own from the
    w x w block of ED_matr it depends on (statistics over the whole series)."""
    Z = znorm_matrix(x, l)
    w = m - l + 1
    out = []
    for s, j in pairs:
        E = ed_matr(Z[s * m: s * m + w], Z[j: j + w])
        out.append(mpd_from_ed(E, k)[0])
    return np.array(out)


def mpdist_pairs_local(x: np.ndarray, m: int, l: int, k: int, pairs) -> np.ndarray:
    """D_s(j) for (s, j) pairs without forming the whole series' z-normalised
    matrix: each of the 2w subsequences involved is z-normalised on its own
    (two-pass, population sigma; the constant threshold uses max |T| of the
    whole series), exactly as znorm_matrix would."""
    x = np.asarray(x, dtype=np.float64)
    thr = const_threshold(x)
    w = m - l + 1

    def z(start):
        W = sliding(x[start: start + w + l - 1], l)
        mu = W.mean(axis=1)
        sig = np.sqrt(((W - mu[:, None]) ** 2).mean(axis=1))
        c = sig <= thr
        Z = (W - mu[:, None]) / np.where(c, 1.0, sig)[:, None]
        Z[c] = 0.0
        return Z

    return np.array([mpd_from_ed(ed_matr(z(s * m), z(j)), k)[0] for s, j in pairs])


def profile_set(x: np.ndarray, m: int, l: int, k: int | None = None,
                segments=None) -> np.ndarray:
    """eq. 15: D = (D_1 .. D_{n/m}), D_s = MPD(S_s, T), shape (nseg, n-m+1)."""
    x = np.asarray(x, dtype=np.float64)
    k = default_k(m) if k is None else k
    nseg = len(x) // m
    w = m - l + 1
    Z = znorm_matrix(x, l)
    segs = range(nseg) if segments is None else segments
    out = []
    for s in segs:
        E = ed_matr(Z[s * m: s * m + w], Z)                  # rows of segment s
        out.append(mpd_from_ed(E, k))
    return np.array(out)


def greedy(D: np.ndarray, K: int):
    """Snippet search of the paper (minimise ProfileArea), done greedily as in
    the original snippets method: each step adds the unchosen segment whose
    profile lowers the area most; ties go to the lowest segment index.
    Returns (picks, areas after each pick)."""
    nseg, Nm = D.shape
    M = np.full(Nm, np.inf)
    picks, areas = [], []
    for _ in range(K):
        best, best_area = -1, np.inf
        for s in range(nseg):
            if s in picks:
                continue
            a = float(np.sum(np.minimum(M, D[s])))
            if a < best_area:
                best, best_area = s, a
        picks.append(best)
        areas.append(best_area)
        M = np.minimum(M, D[best])
    return picks, areas


def neighbours(D: np.ndarray, picks):
    """eqs. 6-7: owner[j] = position in `picks` of the nearest snippet for
    window j (ties to the earliest pick); frac = share of windows owned."""
    P = D[list(picks)]
    owner = np.argmin(P, axis=0)            # argmin returns the first minimum
    Nm = D.shape[1]
    frac = np.array([np.count_nonzero(owner == p) / Nm for p in range(len(picks))])
    return owner, frac


def snippets(x: np.ndarray, m: int, l: int, K: int, k: int | None = None, D=None):
    """The problem statement: the K snippets of length m with index, neighbours
    and frac, ordered by frac descending (eq. 8; stable over greedy order)."""
    if D is None:
        D = profile_set(x, m, l, k)
    picks, areas = greedy(D, K)
    owner, frac = neighbours(D, picks)
    order = sorted(range(K), key=lambda p: -frac[p])
    recs = [dict(segment=int(picks[p]), greedy_rank=p, frac=float(frac[p]),
                 area_after=float(areas[p])) for p in order]
    return dict(records=recs, picks=picks, areas=areas, owner=owner, frac=frac, D=D)


def criterion(D: np.ndarray, picks) -> float:
    """eq. 18 score of one length: sum over ordered pairs p != q of snippets of
    sum_i |D_p(i) - D_q(i)|, divided by the largest entry of D."""
    P = D[list(picks)]
    num = 0.0
    for p in range(len(picks)):
        for q in range(len(picks)):
            if p != q:
                num += float(np.sum(np.abs(P[p] - P[q])))
    den = float(np.max(D))
    return num / den if den > 0 else 0.0


def select_length(x: np.ndarray, m_list, K: int, l_list=None, k_list=None):
    """eq. 18 over the candidate lengths: m_best = argmax score (ties to the smallest m)."""
    scores, results = [], []
    for i, m in enumerate(m_list):
        l = m // 2 if l_list is None else l_list[i]
        k = default_k(m) if k_list is None else k_list[i]
        r = snippets(x, m, l, K, k)
        scores.append(criterion(r["D"], r["picks"]))
        results.append(r)
    best = max(range(len(m_list)), key=lambda i: (scores[i], -m_list[i]))
    return dict(m_best=int(m_list[best]), scores=scores, results=results)


def snippets_multi(X: np.ndarray, m: int, l: int, K: int, k: int | None = None):
    """Snippets of a d-coordinate series X (d x n, eqs. 1-2): section 3.2 runs
    the search on every coordinate independently."""
    X = np.asarray(X, dtype=np.float64)
    assert X.ndim == 2
    return [snippets(X[j], m, l, K, k) for j in range(X.shape[0])]
