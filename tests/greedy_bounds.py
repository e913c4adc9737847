"""Margin-aware comparison of a greedy snippet search against the oracle's.

Section 4.1's greedy step picks the unchosen segment c minimising the area
sum_j min(M_j, D_c(j)) (eqs. 16-17).  Two profile sets that differ entry by
entry (the GPU's FP32 D against the oracle's FP64 D) give areas that differ by
at most

    B_c = sum_j max(|M_gpu(j) - M_ref(j)|, |D_gpu(c, j) - D_ref(c, j)|),

since |min(a, b) - min(a', b')| <= max(|a - a'|, |b - b'|).  So the GPU must
make the oracle's pick b whenever the oracle's margin (second-best area minus
best) exceeds B_b + B_c for the GPU's pick c; otherwise any pick whose oracle
area is within B_b + B_c of the best is a correct outcome of the same method.
Later steps follow the GPU's picks on both sides.
"""
import numpy as np


def _min_curve(D, picks, Nm):
    M = np.full(Nm, np.inf)
    for p in picks:
        M = np.minimum(M, D[p])
    return M


def _area(M, row):
    return float(np.sum(np.minimum(M, row)))


def _bound(Mg, Mr, rg, rr):
    # before the first pick both curves are +inf: no difference there
    both = np.isinf(Mg) & np.isinf(Mr)
    dM = np.abs(np.where(both, 0.0, Mg) - np.where(both, 0.0, Mr))
    return float(np.sum(np.maximum(dM, np.abs(rg - rr))))


def check_greedy(picks_gpu, Dg_rows, Dr_rows, candidates, what=""):
    """picks_gpu: the GPU's picks in greedy order.  Dg_rows / Dr_rows: dicts
    segment -> profile row (float64) for every segment in `candidates` (which
    must hold the GPU's picks).  At each step the oracle's best and runner-up
    among the unchosen candidates are compared with the GPU's pick.  Returns
    one (margin, bound, equal) triple per step."""
    Nm = len(next(iter(Dr_rows.values())))
    out = []
    for t, c in enumerate(picks_gpu):
        chosen = picks_gpu[:t]
        Mg = _min_curve(Dg_rows, chosen, Nm)
        Mr = _min_curve(Dr_rows, chosen, Nm)
        rest = [s for s in candidates if s not in chosen]
        ar = {s: _area(Mr, Dr_rows[s]) for s in rest}
        order = sorted(rest, key=lambda s: (ar[s], s))
        b = order[0]
        margin = ar[order[1]] - ar[b] if len(order) > 1 else float("inf")
        B = _bound(Mg, Mr, Dg_rows[b], Dr_rows[b]) + _bound(Mg, Mr, Dg_rows[c], Dr_rows[c])
        print(f"{what} step {t}: oracle pick {b} margin {margin:.6g}, gpu pick {c}, bound {B:.6g}", flush=True)
        if c != b:
            assert margin <= B, (what, t, b, c, margin, B)
            assert ar[c] - ar[b] <= B, (what, t, b, c, ar[c] - ar[b], B)
        out.append((margin, B, c == b))
    return out


def areas_from_profiles(profiles):
    """ProfileArea after each pick (eq. 17) from the picked profiles in greedy
    order, in FP64."""
    P = np.asarray(profiles, dtype=np.float64)
    M = np.full(P.shape[1], np.inf)
    areas = []
    for row in P:
        M = np.minimum(M, row)
        areas.append(float(np.sum(M)))
    return areas
