"""Write expected snippet results computed by the CPU oracle (oracle/ only).

    python tests/golden/make_golden.py [name ...] [--procs N] [--resume FILE]

Each output file holds the oracle's snippet records, areas, per-step greedy
margins (second-best area minus best) and the runner-up segment of every
step, max D and the eq. 18 score for one named workload built by the seeded
generators.  The sweep workload holds the same for every candidate length and
the length the eq. 18 criterion picks.  The profile set is computed segment
by segment in a process pool (rows written into shared memory).
"""
import json
import os
import sys
from multiprocessing import Pool, resource_tracker, shared_memory

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
SWEEPS = {
    # every candidate length 64, 96, ..., 512 with l = m/2 and K = 6
    "regimes6_n250000_sweep": dict(series=lambda: synth.regime_series(250_000, 3, synth.SHAPES6).x,
                                   m_list=list(range(64, 513, 32)), K=6),
    # the same series with five of those lengths, from the shortest to the
    # longest (the oracle needs about an hour on 7 processes for these five,
    # about five for all fifteen)
    "regimes6_n250000_sweep5": dict(series=lambda: synth.regime_series(250_000, 3, synth.SHAPES6).x,
                                    m_list=[64, 128, 224, 480, 512], K=6),
    # ten of them: every length up to 288, and 480, 512 (about two and a half
    # hours on 7 processes)
    "regimes6_n250000_sweep10": dict(series=lambda: synth.regime_series(250_000, 3, synth.SHAPES6).x,
                                     m_list=[64, 96, 128, 160, 192, 224, 256, 288, 480, 512], K=6),
    # twelve: those ten and 416, 448 (the two take about an hour more)
    "regimes6_n250000_sweep12": dict(series=lambda: synth.regime_series(250_000, 3, synth.SHAPES6).x,
                                     m_list=[64, 96, 128, 160, 192, 224, 256, 288, 416, 448, 480, 512], K=6),
}

_X = None


def _init(x):
    global _X
    _X = x


def _rows(args):
    m, l, k, segs, shm_name, shape = args
    shm = shared_memory.SharedMemory(name=shm_name)
    # the parent owns (and unlinks) the segment
    resource_tracker.unregister(shm._name, "shared_memory")
    try:
        D = np.ndarray(shape, dtype=np.float64, buffer=shm.buf)
        D[segs] = oracle.profile_set(_X, m, l, k, segments=segs)
    finally:
        shm.close()
    return len(segs)


def greedy_margins(D, K):
    """Per greedy step: second-best area minus best, and the second-best segment."""
    nseg = D.shape[0]
    M = np.full(D.shape[1], np.inf)
    chosen, margins, runners = [], [], []
    for _ in range(K):
        areas = np.array([np.inf if s in chosen else float(np.sum(np.minimum(M, D[s])))
                          for s in range(nseg)])
        order = np.argsort(areas, kind="stable")
        if nseg > len(chosen) + 1:
            margins.append(float(areas[order[1]] - areas[order[0]]))
            runners.append(int(order[1]))
        else:
            margins.append(None)
            runners.append(None)
        chosen.append(int(order[0]))
        M = np.minimum(M, D[order[0]])
    return margins, runners


def profile_set_pool(pool, x, m, l, k, procs, use):
    """use(D) on the oracle's profile set of every segment, rows computed in the pool."""
    nseg, Nm = len(x) // m, len(x) - m + 1
    shm = shared_memory.SharedMemory(create=True, size=nseg * Nm * 8)
    try:
        nchunk = max(procs * 4, nseg // 2)  # two segments per task bound a worker's memory
        chunks = [list(range(i, nseg, nchunk)) for i in range(nchunk)]
        chunks = [c for c in chunks if c]
        pool.map(_rows, [(m, l, k, c, shm.name, (nseg, Nm)) for c in chunks], chunksize=1)
        D = np.ndarray((nseg, Nm), dtype=np.float64, buffer=shm.buf)
        out = use(D)
        del D
    finally:
        shm.close()
        shm.unlink()
    return out


def one_length(x, m, l, K, D):
    k = oracle.default_k(m)
    r = oracle.snippets(x, m, l, K, k, D=D)
    margins, runners = greedy_margins(D, K)
    return dict(
        n=len(x), m=m, l=l, k=k, K=K,
        records=r["records"], picks=[int(p) for p in r["picks"]],
        areas=[float(a) for a in r["areas"]], margins=margins, runners=runners,
        counts=[int(np.count_nonzero(r["owner"] == p)) for p in range(K)],
        dmax=float(D.max()), score=oracle.criterion(D, r["picks"]),
    )


def make(name, procs=8):
    c = CASES[name]
    x = c["series"]()
    m, l, K = c["m"], c["l"], c["K"]
    with Pool(procs, initializer=_init, initargs=(x,)) as pool:
        res = profile_set_pool(pool, x, m, l, oracle.default_k(m), procs,
                               lambda D: one_length(x, m, l, K, D))
    out = dict(workload=name, **res,
               source="oracle.snippets on the seeded generator (tests/golden/make_golden.py)")
    with open(os.path.join(HERE, f"snippets_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def make_sweep(name, procs=8, resume=None):
    """resume: a JSON-lines file that keeps each finished length, so that an
    interrupted run continues where it stopped."""
    c = SWEEPS[name]
    x = c["series"]()
    K = c["K"]
    path = os.path.join(HERE, f"sweep_{name}.json")
    done = {}
    if resume and os.path.exists(resume):
        for line in open(resume):
            r = json.loads(line)
            done[r["m"]] = r
    # longest lengths first: they take the most memory and time
    todo = sorted((m for m in c["m_list"] if m not in done), reverse=True)
    with Pool(procs, initializer=_init, initargs=(x,), maxtasksperchild=16) as pool:
        for m in todo:
            l = m // 2
            done[m] = profile_set_pool(pool, x, m, l, oracle.default_k(m), procs,
                                       lambda D: one_length(x, m, l, K, D))
            print(name, "m", m, "picks", done[m]["picks"], "score", done[m]["score"], flush=True)
            if resume:
                with open(resume, "a") as f:
                    f.write(json.dumps(done[m]) + "\n")
    per = [done[m] for m in c["m_list"]]
    scores = [p["score"] for p in per]
    ms = [p["m"] for p in per]
    # eq. 18: the largest score, ties to the smallest m (as oracle.select_length)
    best = max(range(len(ms)), key=lambda i: (scores[i], -ms[i]))
    out = dict(workload=name, n=len(x), K=K, m_list=ms, scores=scores, m_best=ms[best],
               lengths=per,
               source="oracle.snippets and oracle.criterion per length on the seeded generator "
                      "(tests/golden/make_golden.py)")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    procs, resume = 8, None
    if "--procs" in args:
        i = args.index("--procs")
        procs = int(args[i + 1])
        del args[i:i + 2]
    if "--resume" in args:
        i = args.index("--resume")
        resume = args[i + 1]
        del args[i:i + 2]
    for name in args or list(CASES):
        if name in SWEEPS:
            o = make_sweep(name, procs, resume)
            print(name, "m_best", o["m_best"], flush=True)
        else:
            o = make(name, procs)
            print(name, o["picks"], o["margins"], o["runners"], flush=True)
