"""Write expected snippet results computed by the CPU oracle (oracle/ only).

    python tests/golden/make_golden.py [name ...]

Each output file holds the oracle's snippet records, areas, per-step greedy
margins (second-best area minus best), max D and the eq. 18 score for one named
workload built by the seeded generators.  The profile set is computed
segment by segment in a process pool.
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2401_13680_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    "four_regimes_n2000": dict(series=lambda: synth.four_regimes(1).x, m=100, l=50, K=3),
    "regimes5_n100000": dict(series=lambda: synth.regime_series(100_000, 2, synth.SHAPES5).x,
                             m=256, l=128, K=4),
}

_X = None


def _init(x):
    global _X
    _X = x


def _rows(args):
    m, l, k, segs = args
    return oracle.profile_set(_X, m, l, k, segments=segs)


def greedy_margins(D, K):
    nseg = D.shape[0]
    M = np.full(D.shape[1], np.inf)
    chosen, margins = [], []
    for _ in range(K):
        areas = np.array([np.inf if s in chosen else float(np.sum(np.minimum(M, D[s])))
                          for s in range(nseg)])
        order = np.argsort(areas, kind="stable")
        margins.append(float(areas[order[1]] - areas[order[0]]) if nseg > len(chosen) + 1 else None)
        chosen.append(int(order[0]))
        M = np.minimum(M, D[order[0]])
    return margins


def make(name, procs=8):
    c = CASES[name]
    x = c["series"]()
    m, l, K = c["m"], c["l"], c["K"]
    k = oracle.default_k(m)
    nseg = len(x) // m
    chunks = [list(range(i, nseg, procs * 4)) for i in range(procs * 4)]
    with Pool(procs, initializer=_init, initargs=(x,)) as pool:
        parts = pool.map(_rows, [(m, l, k, ch) for ch in chunks if ch])
    D = np.empty((nseg, len(x) - m + 1))
    for ch, part in zip([ch for ch in chunks if ch], parts):
        D[ch] = part
    r = oracle.snippets(x, m, l, K, k, D=D)
    out = dict(
        workload=name, n=len(x), m=m, l=l, k=k, K=K,
        records=r["records"], picks=[int(p) for p in r["picks"]],
        areas=[float(a) for a in r["areas"]], margins=greedy_margins(D, K),
        counts=[int(np.count_nonzero(r["owner"] == p)) for p in range(K)],
        dmax=float(D.max()), score=oracle.criterion(D, r["picks"]),
        source="oracle.snippets on the seeded generator (tests/golden/make_golden.py)",
    )
    with open(os.path.join(HERE, f"snippets_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        o = make(name)
        print(name, o["picks"], o["margins"])
