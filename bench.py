"""Benchmark: MPdist distance-matrix cells per second on one MI355X, with
p50/p99 request latency.

Default workload (the metric's own): the serving stream of regime-switching
series, Poisson arrivals at 20 requests/s, n log-uniform in [1e4, 5e5], m
uniform in {64, 128, 256, 512, 1024}, l = m/2, K uniform in 3..5.  A step is
ten requests of the stream, so --steps 20 serves the 200-request stream.
Inputs are resident in HBM (pst_submit_device) when the timed region starts.
The whole stream (all steps' requests) is submitted at once and served with
continuous batching; `value` = its distance-matrix cells / the time to serve
it, and ms_per_step = that time / steps.  The plain per-request path
(pst_snippets one request after another) is measured beside it; p50/p99 come
from a replay at the stream's own arrival times.
cells = nseg * (m-l+1) * (n-l+1) per request.

--workload plain: one 100 000-point five-shape series, m=256, l=128, K=4, the
whole snippet search per step.  Other workloads: sweep, multi, schedule,
blocked, probe.

Prints one JSON line.  --gpus N with N > 1 is refused: the library drives one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="regimes5_n100000", n=100_000, m=256, l=128, K=4)
# Algorithmic VALU lane-operations per distance-matrix cell (see the design
# notes): covariance update 2 FMA, correlation 2 MUL, column max 1, sliding
# row max 1, k-th selection 2 (each cell feeds 2 of the 2w values per window).
OPS_PER_CELL = 8
# 256 CUs x 64 lanes x 2.4 GHz: VALU lane-operations per second (non-packed).
PEAK_LANE_OPS = 256 * 64 * 2.4e9


TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "k_profile_traffic.md")
KERNEL_HASH = os.path.join(ROOT, "paper_2401_13680_amd", "libpst.k_profile.sha256")


def progress(msg):
    """A progress line on stderr (the JSON result stays the last line of stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(cells_per_launch, field="hbm bytes per cell"):
    """HBM bytes per profile launch: the committed FETCH_SIZE + WRITE_SIZE
    measurement (bytes per distance-matrix cell, copy-calibrated) times the
    launch's cells, or None once the profile kernel's machine code differs from
    the one measured (hash written by the build)."""
    try:
        note = open(TRAFFIC_NOTE).read()
        built = open(KERNEL_HASH).read().strip()
    except OSError:
        return None
    fields = {}
    for line in note.splitlines():
        if ":" in line and line.startswith("- "):
            key, _, val = line[2:].partition(":")
            fields[key.strip()] = val.strip().strip("`")
    if fields.get("k_profile code sha256") != built or field not in fields:
        return None
    return float(fields[field]) * cells_per_launch


def cpu_baseline(x, m, l, k, nseg_sample=20):
    """The FP64 oracle on a bounded sample of segments of the same workload."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    n = len(x)
    w = m - l + 1
    segs = list(range(0, n // m, max(1, (n // m) // nseg_sample)))[:nseg_sample]
    t0 = time.perf_counter()
    oracle.profile_set(x, m, l, k, segments=segs)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    cells = len(segs) * w * (n - l + 1)
    return dict(value=cells / dt, unit="cells/s", cores=1, kind="oracle",
                sample=f"profiles of {len(segs)} of {n // m} segments ({cells:.3g} cells, "
                       f"{dt:.1f} s), numpy FP64, BLAS limited to 1 thread")


PROBE_NAMES = {0: "windows", 1: "run_starts", 2: "windows_by_own_pass", 3: "cooperative_selects",
               4: "misses_below", 5: "misses_above", 6: "list_overflows", 7: "misses_at_run_start",
               8: "overflows_of_one_key_brackets", 9: "sum_of_list_lengths", 10: "overflows_holding_kth",
               11: "second_pass_brackets", 12: "windows_by_second_pass"}
PROBE_PHASES = {16: "distance phase", 17: "  FP64 anchors", 18: "  FP32 recurrence", 19: "  column minima",
                20: "  sliding row minima", 21: "selection phase", 22: "  run starts (radix select)",
                23: "  bracket passes", 24: "  sorts and second passes", 25: "  cooperative selects"}


def probe_bench(args):
    """Phase split of the profile kernel on the 100 000-point workload from the
    probe build (libpst_probe.so, built by `python -m paper_2401_13680_amd.build
    --probe`): wave cycles per phase and how often the selection's paths run.
    The probe's own atomics slow the kernel; the split, not the time, is the
    result."""
    import ctypes

    import torch

    from paper_2401_13680_amd import _lib, api, synth

    _lib.LIB_PATH = _lib.PROBE_LIB_PATH
    L = _lib.load()
    L.pst_probe_read.argtypes = [ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int]
    buf = (ctypes.c_ulonglong * 32)()
    m = args.probe_m or WORKLOAD["m"]
    l = m // 2
    T = torch.from_numpy(synth.workload_series(WORKLOAD["name"])).cuda()
    if args.probe_geometry:
        api.set_geometry(m - l + 1, int(args.probe_geometry, 0))
    api.profile_set(T, m, l)
    torch.cuda.synchronize()
    L.pst_probe_read(buf, 1)
    api.profile_set(T, m, l)
    torch.cuda.synchronize()
    L.pst_probe_read(buf, 1)
    tot = buf[16] + buf[21]
    out = dict(workload=WORKLOAD["name"], m=m, l=l, geometry=hex(api.geometry(m - l + 1)), counts={v: int(buf[k]) for k, v in PROBE_NAMES.items()},
               wave_cycles={v.strip(): int(buf[k]) for k, v in PROBE_PHASES.items()},
               share_of_wave_time={v.strip(): round(buf[k] / tot, 4) for k, v in PROBE_PHASES.items()})
    print(json.dumps(out), flush=True)


def geometry_bench(args):
    """Every tile geometry of the profile kernel, per m of the serving stream
    (m in {64, .., 1024}, l = m/2): all segment profiles of a 200 000-point
    five-shape series, three launches each after a warm-up, against the
    built-in choice and the tuner's."""
    import torch

    from paper_2401_13680_amd import api, synth

    n = 200_000
    out = {}
    for m in (64, 128, 256, 512, 1024):
        l = m // 2
        w = m - l + 1
        T = torch.from_numpy(synth.regime_series(n, 70 + m, len_range=(2000, 8000)).x).cuda()

        def t_profile():
            api.profile_set(T, m, l)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                api.profile_set(T, m, l)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / 3 * 1e3

        base = t_profile()
        res = {}
        for code in api.geometry_candidates(w):
            api.set_geometry(w, code)
            res[hex(code)] = round(t_profile(), 2)
        api.set_geometry(w, 0)
        code, _ = api.tune_geometry(T, m, l)
        tuned = t_profile()
        api.set_geometry(w, 0)
        cells = (n // m) * w * (n - l + 1)
        out[m] = dict(w=w, builtin=hex(api.geometry(w)), builtin_ms=round(base, 2), tuned=hex(code),
                      tuned_ms=round(tuned, 2), all_ms=res, builtin_cells_per_s=cells / base * 1e3)
        progress(f"m={m}: built-in {base:.1f} ms, tuned {tuned:.1f} ms")
    print(json.dumps(dict(workload="geometries_regimes5_n200000", per_m=out)), flush=True)


def sweep_bench(args):
    """Length sweep: 250 000-point six-shape series, m in {64, 96, .., 512},
    l = m/2, K = 6; batched + graph against one length at a time."""
    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    n, ms, K = 250_000, list(range(64, 513, 32)), 6
    x = synth.workload_series("regimes6_n250000_sweep")
    T = torch.from_numpy(x).cuda()
    cells = sum((n // m) * (m - m // 2 + 1) * (n - m // 2 + 1) for m in ms)
    res = {}
    modes = [("batched_graph", dict(batched=True, graph=True)), ("plain", dict(batched=False)),
             ("batched_graph_one_launch", dict(batched=True, graph=True, one_launch=True))]
    if not args.no_tune:
        modes.append(("batched_graph_tuned", dict(batched=True, graph=True, tune_geometry=True)))
    for mode, kw in modes:
        progress(f"sweep mode {mode}")
        for _ in range(args.warmup):
            api.select_length(T, ms, K, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = api.select_length(T, ms, K, **kw)
        torch.cuda.synchronize()
        res[mode] = (time.perf_counter() - t0) / args.steps, r["m_best"]
    dt, mb = res["batched_graph"]
    # labelling of the series by the snippets of the chosen length, scored by
    # per-element F1 against the generator's regime labels (section 5.2)
    S = synth.regime_series(n, 3, synth.SHAPES6)
    r = api.select_length(T, ms, K, owner=True)
    truth = torch.from_numpy(S.labels.astype(np.int32)).cuda()
    C = int(S.labels.max()) + 1
    lab = api.label_f1(r["owner"], truth, r["m_best"], K, C)
    out = dict(metric="MPdist distance-matrix cells/sec on 1 MI355X; p50/p99 request latency",
               value=cells / dt, unit="cells/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=dt * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload="regimes6_n250000_sweep", n=n, m_list=ms, l="m/2", K=K,
                           cells_per_step=cells, m_best=mb,
                           step="all 15 lengths: stats + profiles in one launch + greedy + criterion, one HIP graph"),
               plain_one_length_at_a_time=dict(value=cells / res["plain"][0], ms_per_step=res["plain"][0] * 1e3),
               batched_over_plain=res["plain"][0] / dt,
               one_launch_all_lengths=dict(value=cells / res["batched_graph_one_launch"][0],
                                           ms_per_step=res["batched_graph_one_launch"][0] * 1e3,
                                           m_best=res["batched_graph_one_launch"][1],
                                           per_shape_over_one_launch=res["batched_graph_one_launch"][0] / dt),
               tuned_geometries=(dict(value=cells / res["batched_graph_tuned"][0],
                                      ms_per_step=res["batched_graph_tuned"][0] * 1e3,
                                      m_best=res["batched_graph_tuned"][1],
                                      over_builtin=dt / res["batched_graph_tuned"][0],
                                      geometry={str(m): hex(api.geometry(m - m // 2 + 1)) for m in ms})
                                 if "batched_graph_tuned" in res else None),
               labelling=dict(m_best=r["m_best"], classes=C, macro_f1=lab["macro_f1"],
                              f1=[round(v, 4) for v in lab["f1"]]))
    print(json.dumps(out), flush=True)


def multi_bench(args):
    """Multivariate: 4 coordinates of 100 000 points switching regime together,
    m=256, l=128, K=4 per coordinate; every coordinate's profiles in one
    launch against one coordinate after another."""
    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    wl = synth.WORKLOADS["multi4_n100000"]
    n, d, m, l, K = wl["n"], wl["d"], wl["m"], wl["l"], wl["K"]
    S = synth.multivariate_series(n, d, 6)
    X = torch.from_numpy(S.x).cuda()
    cells = d * (n // m) * (m - l + 1) * (n - l + 1)
    res = {}
    for mode in ("batched", "plain"):
        def step():
            if mode == "batched":
                return api.snippets_multi(X, m, l, K, owner=True)
            return [api.snippets(X[j], m, l, K, owner=True) for j in range(d)]
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = step()
        torch.cuda.synchronize()
        res[mode] = ((time.perf_counter() - t0) / args.steps, r)
    dt, r = res["batched"]
    same = all(r[j]["records"] == res["plain"][1][j]["records"] for j in range(d))
    truth = torch.from_numpy(S.labels.astype(np.int32)).cuda()
    C = int(S.labels.max()) + 1
    f1 = [api.label_f1(r[j]["owner"], truth, m, K, C)["macro_f1"] for j in range(d)]
    out = dict(metric="MPdist distance-matrix cells/sec on 1 MI355X; p50/p99 request latency",
               value=cells / dt, unit="cells/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=dt * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload="multi4_n100000", n=n, d=d, m=m, l=l, K=K, cells_per_step=cells,
                           step="stats of every coordinate + all profiles in one launch + greedy + neighbours"),
               plain_one_coordinate_at_a_time=dict(value=cells / res["plain"][0], ms_per_step=res["plain"][0] * 1e3),
               batched_over_plain=res["plain"][0] / dt, batched_equals_plain=same,
               labelling=dict(classes=C, macro_f1_per_coordinate=[round(v, 4) for v in f1]))
    print(json.dumps(out), flush=True)


def schedule_bench(args):
    """Scheduling of section 4.2 on measured run times: a polynomial model fitted
    on plain per-length runs of three training series predicts the run times of
    the 15 lengths of the sweep workload (held out); the lengths are then spread
    over P workers by Karmarkar-Karp on the predictions, and each worker's
    measured load is compared with contiguous and round-robin splits."""
    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    K = 4

    def run_ms(T, m):
        api.snippets(T, m, m // 2, K)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(max(args.steps, 1)):
            t0 = time.perf_counter()
            api.snippets(T, m, m // 2, K)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) * 1e3)
        return best

    train = []
    for n, seed in ((60_000, 31), (120_000, 32), (180_000, 33)):
        T = torch.from_numpy(synth.regime_series(n, seed, synth.SHAPES6).x).cuda()
        for m in range(64, 513, 64):
            train.append((n, m, m // 2, run_ms(T, m)))
    n = 250_000
    ms_list = list(range(64, 513, 32))
    T = torch.from_numpy(synth.workload_series("regimes6_n250000_sweep")).cuda()
    actual = [run_ms(T, m) for m in ms_list]
    out = dict(workload="schedule_regimes6_n250000", train_runs=len(train), held_out=len(ms_list), models={})
    for D in (1, 2, 3):
        M = api.RuntimeModel(D)
        for r in train:
            M.observe(*r)
        M.fit()
        pred = [M.predict(n, m, m // 2) for m in ms_list]
        rel = [abs(p - a) / a for p, a in zip(pred, actual)]
        splits = {}
        for P in (2, 4, 8):
            part, _ = api.partition_lengths(M, n, ms_list, P)
            def imb(assign):
                loads = [sum(a for a, q in zip(actual, assign) if q == j) for j in range(P)]
                return max(loads) / (sum(loads) / P)
            contiguous = [min(i * P // len(ms_list), P - 1) for i in range(len(ms_list))]
            round_robin = [i % P for i in range(len(ms_list))]
            splits[f"P{P}"] = dict(kk=round(imb(part), 4), contiguous=round(imb(contiguous), 4),
                                   round_robin=round(imb(round_robin), 4))
        out["models"][f"degree{D}"] = dict(mean_rel_err=round(float(np.mean(rel)), 4),
                                           max_rel_err=round(float(np.max(rel)), 4),
                                           max_load_over_mean=splits)
    out["actual_ms"] = [round(a, 3) for a in actual]
    print(json.dumps(out), flush=True)


def blocked_bench(args):
    """Bounded memory: a 10^6-point five-shape series, m=256, l=128, K=4 (profile
    set 15.6 GB), in core against pst_snippets_blocked with a 4 GiB workspace, and
    against pst_snippets_spilled (the same workspace, D kept in pinned host memory)."""
    import torch

    from paper_2401_13680_amd import api, synth

    n, m, l, K = 1_000_000, 256, 128, 4
    T = torch.from_numpy(synth.regime_series(n, 8, synth.SHAPES5).x).cuda()
    cells = (n // m) * (m - l + 1) * (n - l + 1)
    res = {}
    D_host = torch.empty((n // m, n - m + 1), dtype=torch.float32, pin_memory=True)
    for mode in ("in_core", "blocked", "spilled"):
        def step():
            if mode == "in_core":
                return api.snippets(T, m, l, K, owner=True)
            if mode == "blocked":
                return api.snippets_blocked(T, m, l, K, budget_bytes=4 << 30, owner=True)
            return api.snippets_spilled(T, m, l, K, budget_bytes=4 << 30, D_host=D_host, owner=True)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(args.steps, 1)):
            r = step()
        torch.cuda.synchronize()
        res[mode] = ((time.perf_counter() - t0) / max(args.steps, 1), r)
    ctx = api.context(0)
    ws_in = int(ctx.L.pst_workspace_bytes(n, m, l, K))
    rb = res["blocked"][1]
    out = dict(workload="blocked_regimes5_n1000000", n=n, m=m, l=l, K=K, cells=cells,
               in_core=dict(seconds=round(res["in_core"][0], 4), workspace_bytes=ws_in,
                            cells_per_s=cells / res["in_core"][0]),
               blocked=dict(seconds=round(res["blocked"][0], 4), workspace_bytes=rb["workspace_bytes"],
                            seg_block=rb["seg_block"], segments=n // m,
                            cells_per_s_of_the_problem=cells / res["blocked"][0]),
               spilled=dict(seconds=round(res["spilled"][0], 4), workspace_bytes=res["spilled"][1]["workspace_bytes"],
                            host_bytes=D_host.numel() * 4, cells_per_s_of_the_problem=cells / res["spilled"][0],
                            identical=res["spilled"][1]["records"] == res["in_core"][1]["records"]),
               time_ratio=res["blocked"][0] / res["in_core"][0],
               memory_ratio=ws_in / rb["workspace_bytes"],
               identical=(rb["records"] == res["in_core"][1]["records"]
                          and bool(torch.equal(rb["owner"], res["in_core"][1]["owner"]))))
    print(json.dumps(out), flush=True)


def _cpu_task(args):
    import numpy as np
    import oracle
    x, m, l, s = args
    t0 = time.perf_counter()
    oracle.profile_set(np.asarray(x), m, l, None, segments=[s])
    return time.perf_counter() - t0


def cpu_baseline_serving(reqs, per_m=4, n_max=150_000):
    """The FP64 oracle on a bounded sample of the serving stream: the middle
    segment of the first `per_m` requests of each m with n <= n_max, on a
    process pool over every host core, and three of them on one core."""
    import platform
    from multiprocessing import get_context

    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        pass
    cores = len(os.sched_getaffinity(0))
    tasks, seen = [], {}
    for r in reqs:
        if len(r.x) <= n_max and seen.get(r.m, 0) < per_m:
            seen[r.m] = seen.get(r.m, 0) + 1
            tasks.append((r.x, r.m, r.l, (len(r.x) // r.m) // 2))
    cells = [(len(x) - l + 1) * (m - l + 1) for x, m, l, _ in tasks]
    env = dict(OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        with get_context("spawn").Pool(min(cores, len(tasks))) as pool:
            t0 = time.perf_counter()
            pool.map(_cpu_task, tasks, chunksize=1)
            wall = time.perf_counter() - t0
        firsts = [next(i for i, t in enumerate(tasks) if t[1] == m) for m in sorted({t[1] for t in tasks})]
        one = [_cpu_task(tasks[i]) for i in firsts]
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    try:
        model = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")][0]
    except Exception:  # pragma: no cover
        model = platform.processor()
    return dict(value=sum(cells) / wall, unit="cells/s", cores=min(cores, len(tasks)), kind="oracle",
                sample=f"profile of the middle segment of {len(tasks)} requests of the stream ({per_m} per m, "
                       f"n <= {n_max}; {sum(cells):.3g} cells, {wall:.1f} s) on a process pool, numpy FP64, "
                       f"BLAS 1 thread per process",
                one_core=dict(value=sum(cells[i] for i in firsts) / sum(one), unit="cells/s",
                              sample=f"one of those segments per m ({len(firsts)}), {sum(one):.1f} s"),
                host=dict(nproc=os.cpu_count(), affinity=cores, cpu=model))


def serve_bench(args):
    """The serving stream (the metric's workload): Poisson arrivals (20/s) of
    regime-switching series, n log-uniform in [1e4, 5e5], m in {64, .., 1024},
    l = m/2, K in 3..5; ten requests per step."""
    import ctypes

    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    nreq = 10 * args.steps
    reqs = synth.poisson_requests(num=nreq, rate=20.0, seed=5)
    warm = synth.poisson_requests(num=10 * args.warmup, rate=20.0, seed=105) if args.warmup > 0 else []
    cells_of = lambda r: (len(r.x) // r.m) * (r.m - r.l + 1) * (len(r.x) - r.l + 1)
    cells = sum(cells_of(r) for r in reqs)
    Ts = [torch.from_numpy(r.x).cuda() for r in reqs]
    Tw = [torch.from_numpy(r.x).cuda() for r in warm]
    torch.cuda.synchronize()
    budget, slots = 160 << 30, 32
    # tile geometry of each m of the stream, tuned on a series of the same
    # generator that is not part of the stream (both paths below use it)
    geometry = {}
    progress(f"{nreq} requests, {cells:.3g} cells; tuning tile geometries")
    if not args.no_tune:
        for m in sorted({r.m for r in reqs}):
            xt = synth.regime_series(200_000, 900 + m, synth.SHAPES5).x
            code, _ = api.tune_geometry(torch.from_numpy(xt).cuda(), m, m // 2)
            geometry[str(m)] = api.decode_geometry(code)
    if args.plain_only:  # the plain pass alone (for profiler runs of its profile launches)
        progress("plain pass")
        ctx = api.context(0)
        for T, r in zip(Tw[:3], warm[:3]):
            api.snippets(T, r.m, r.l, r.K, ctx=ctx)
        torch.cuda.synchronize()
        ctx.L.pst_set_timing(ctx.h, 1)
        kms, ms = [], ctypes.c_float()
        for T, r in zip(Ts, reqs):
            api.snippets(T, r.m, r.l, r.K, ctx=ctx)
            ctx.check(ctx.L.pst_last_profile_ms(ctx.h, ctypes.byref(ms)))
            kms.append(ms.value)
        torch.cuda.synchronize()
        ctx.L.pst_set_timing(ctx.h, 0)
        if args.calibrate_copy:  # one 1 GiB device copy: the counters' reading for known bytes
            a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            torch.cuda.synchronize()
            b.copy_(a)
            torch.cuda.synchronize()
        print(json.dumps(dict(workload=f"poisson20_serving_{nreq}", plain_only=True, cells=cells,
                              profile_launches=nreq, kernel_ms=float(np.mean(kms)),
                              launch_m=[r.m for r in reqs], launch_cells=[cells_of(r) for r in reqs],
                              tile_geometry_by_m={m: hex(api.geometry(m - m // 2 + 1))
                                                  for m in sorted({r.m for r in reqs})})), flush=True)
        return

    def serve_all(srv, series, rs):
        tk = [srv.submit(T, r.m, r.l, r.K) for T, r in zip(series, rs)]
        srv.drain()
        return [srv.poll(t) for t in tk]

    progress("served pass")
    srv = api.Server(0, hbm_budget_bytes=budget, max_slots=slots)
    if warm:
        serve_all(srv, Tw, warm)
    b0 = srv.stats()["batches"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    served = serve_all(srv, Ts, reqs)
    sat = time.perf_counter() - t0
    nbatch = srv.stats()["batches"] - b0
    assert all(r["status"] == 0 for r in served)

    # plain: pst_snippets one request after another, the profile kernel timed
    # by the library's events around each launch
    progress("plain pass")
    ctx = api.context(0)
    L = ctx.L
    for T, r in zip(Tw[:3], warm[:3]):
        api.snippets(T, r.m, r.l, r.K, ctx=ctx)
    torch.cuda.synchronize()
    L.pst_set_timing(ctx.h, 1)
    kms, ms = [], ctypes.c_float()
    t0 = time.perf_counter()
    plain_recs = []
    for T, r in zip(Ts, reqs):
        plain_recs.append(api.snippets(T, r.m, r.l, r.K, ctx=ctx)["records"])
        ctx.check(L.pst_last_profile_ms(ctx.h, ctypes.byref(ms)))
        kms.append(ms.value)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    L.pst_set_timing(ctx.h, 0)
    same = all(a["records"] == b for a, b in zip(served, plain_recs))

    # latency: the stream replayed at its own arrival times
    progress("Poisson replay")
    t0 = time.perf_counter()
    tickets = []
    for T, r in zip(Ts, reqs):
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(T, r.m, r.l, r.K))
    srv.drain()
    span = time.perf_counter() - t0
    lat = [srv.poll(t)["latency_ms"] for t in tickets]
    srv.close()

    # the same stream submitted from host memory (PCIe copies included)
    progress("host-memory submissions")
    srv = api.Server(0, hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()
    serve_all(srv, [r.x for r in reqs], reqs)
    host_sat = time.perf_counter() - t0
    srv.close()

    k_ms = float(np.sum(kms))
    achieved = OPS_PER_CELL * cells / (k_ms * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    offered = cells / reqs[-1].arrival_s
    per_m = {}
    for r, t in zip(reqs, kms):
        a = per_m.setdefault(r.m, [0.0, 0.0, 0])
        a[0] += cells_of(r)
        a[1] += t
        a[2] += 1
    kernel_by_m = {str(m): dict(requests=a[2], cells_per_s=a[0] / (a[1] * 1e-3), geometry=hex(api.geometry(m - m // 2 + 1)))
                   for m, a in sorted(per_m.items())}
    out = dict(metric="MPdist distance-matrix cells/sec on 1 MI355X; p50/p99 request latency",
               value=cells / sat, unit="cells/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=sat * 1e3 / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload=f"poisson20_serving_{nreq}", requests=nreq, requests_per_step=10,
                           n="log-uniform [1e4, 5e5]", m=[64, 128, 256, 512, 1024], l="m/2", K="3..5",
                           rate_per_s=20.0, cells=cells,
                           step="ten requests' share of the stream: all the steps' requests are submitted "
                                "at once with series in HBM and served with continuous batching; "
                                "ms_per_step is their time over the steps"),
               latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                               mean=float(np.mean(lat)), replay_s=span,
                               offered_cells_per_s=offered,
                               offered_over_capacity=offered / (cells / sat)),
               plain_one_request_at_a_time=dict(value=cells / plain, seconds=plain),
               served_over_plain=plain / sat, served_equals_plain=same, batches=nbatch,
               host_submit_pcie_inclusive=dict(value=cells / host_sat, seconds=host_sat),
               roofline=dict(bound="alu", achieved=achieved, peak=peak, unit="Tops/s (VALU lane-ops)",
                             frac=achieved / peak, traffic=measured_traffic(cells_per_launch=cells / nreq),
                             kernel="k_profile", kernel_ms=k_ms / nreq, launches=nreq,
                             ops_per_cell=OPS_PER_CELL,
                             note="profile launches of the plain pass over the same requests, "
                                  "HIP events around each launch"),
               profile_kernel_by_m=kernel_by_m, tile_geometry_by_m=geometry or "built-in")
    if not args.no_cpu_baseline:
        progress("CPU baseline")
        out["cpu_baseline"] = cpu_baseline_serving(reqs)
    print(json.dumps(out), flush=True)


def serve_order_bench(args):
    """Admission order under queueing: the serving stream replayed with two
    slots, in arrival order and shortest predicted first (run-time model of
    section 4.2 seeded with the plain per-request times)."""
    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    reqs = synth.poisson_requests(num=args.requests, rate=20.0, seed=5)
    Ts = [torch.from_numpy(r.x).cuda() for r in reqs]
    api.snippets(Ts[0], reqs[0].m, reqs[0].l, reqs[0].K)
    model = api.RuntimeModel(2)
    for r, T in zip(reqs, Ts):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        api.snippets(T, r.m, r.l, r.K)
        torch.cuda.synchronize()
        model.observe(len(r.x), r.m, r.l, (time.perf_counter() - t1) * 1e3)
    model.fit()
    order = {}
    for name, pol in (("arrival", api.Server.ARRIVAL), ("shortest_predicted_first", api.Server.SHORTEST_PREDICTED)):
        srv = api.Server(0, hbm_budget_bytes=96 << 30, max_slots=2)
        srv.set_policy(pol, model if pol else None)
        t0 = time.perf_counter()
        tickets = []
        for T, r in zip(Ts, reqs):
            delay = r.arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(T, r.m, r.l, r.K))
        srv.drain()
        sp = time.perf_counter() - t0
        lt = [srv.poll(t)["latency_ms"] for t in tickets]
        srv.close()
        order[name] = dict(seconds=round(sp, 4), p50=round(float(np.percentile(lt, 50)), 2),
                           p99=round(float(np.percentile(lt, 99)), 2), mean=round(float(np.mean(lt)), 2))
    print(json.dumps(dict(workload=f"poisson20_serving_{len(reqs)}_two_slots", admission_order=order)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="serve",
                    choices=["serve", "plain", "serve_order", "sweep", "multi", "schedule", "blocked", "probe",
                             "geometry"])
    ap.add_argument("--requests", type=int, default=40, help="serve_order: number of requests")
    ap.add_argument("--probe-m", type=int, default=0, help="probe: snippet length (l = m/2)")
    ap.add_argument("--probe-geometry", default="", help="probe: tile geometry code to install first")
    ap.add_argument("--no-tune", action="store_true", help="serve, sweep: keep the built-in tile geometries")
    ap.add_argument("--plain-only", action="store_true",
                    help="serve: only the plain per-request pass (one profile launch per request)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one 1 GiB device copy (reference for FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py drives exactly one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "sweep":
        return sweep_bench(args)
    if args.workload == "serve":
        return serve_bench(args)
    if args.workload == "serve_order":
        return serve_order_bench(args)
    if args.workload == "multi":
        return multi_bench(args)
    if args.workload == "schedule":
        return schedule_bench(args)
    if args.workload == "blocked":
        return blocked_bench(args)
    if args.workload == "probe":
        return probe_bench(args)
    if args.workload == "geometry":
        return geometry_bench(args)

    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    n, m, l, K = WORKLOAD["n"], WORKLOAD["m"], WORKLOAD["l"], WORKLOAD["K"]
    k = synth.default_k(m)
    w = m - l + 1
    nseg = n // m
    cells = nseg * w * (n - l + 1)
    x = synth.workload_series(WORKLOAD["name"])
    T = torch.from_numpy(x).cuda()
    ctx = api.context(0)
    L = ctx.L

    for _ in range(args.warmup):
        api.snippets(T, m, l, K, k, ctx=ctx)
    torch.cuda.synchronize()
    L.pst_set_timing(ctx.h, 1)
    lat, kms = [], []
    import ctypes
    ms = ctypes.c_float()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        api.snippets(T, m, l, K, k, ctx=ctx)
        lat.append((time.perf_counter() - s0) * 1e3)
        ctx.check(L.pst_last_profile_ms(ctx.h, ctypes.byref(ms)))
        kms.append(ms.value)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.pst_set_timing(ctx.h, 0)

    ms_step = dt * 1e3 / args.steps
    value = cells / (dt / args.steps)
    k_ms = float(np.mean(kms))
    achieved = OPS_PER_CELL * cells / (k_ms * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    out = dict(
        metric="MPdist distance-matrix cells/sec on 1 MI355X; p50/p99 request latency",
        value=value, unit="cells/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD["name"], n=n, m=m, l=l, k=k, K=K, cells_per_step=cells,
                    step="stats + all segment profiles + greedy + neighbours"),
        latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99))),
        roofline=dict(bound="alu", achieved=achieved, peak=peak, unit="Tops/s (VALU lane-ops)",
                      frac=achieved / peak, traffic=measured_traffic(cells, "hbm bytes per cell at m=256"), kernel="k_profile",
                      kernel_ms=k_ms, ops_per_cell=OPS_PER_CELL),
    )
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, m, l, k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
