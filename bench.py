"""Benchmark: MPdist distance-matrix cells per second on one MI355X.

One step = the whole snippet-finding hot path on one series, resident in HBM:
FP64 window statistics, the MPdist profile of every segment (eqs. 9-15), the
greedy minimum-area snippet search, neighbours and frac (eqs. 6-8, 16-17).
Workload: 100 000-point regime-switching series of 5 shapes, m=256, l=128,
k=26, K=4.  cells = nseg * (m-l+1) * (n-l+1) distance-matrix entries.

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


TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "k_profile_regimes5_n100000_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2401_13680_amd", "csrc", "pst_profile.hip")


def measured_traffic():
    """HBM bytes per profile launch from the committed FETCH_SIZE / WRITE_SIZE
    measurement, or None once the kernel source differs from the one measured."""
    import hashlib
    try:
        note = open(TRAFFIC_NOTE).read()
    except OSError:
        return None
    fields = {}
    for line in note.splitlines():
        if ":" in line and line.startswith("- "):
            key, _, val = line[2:].partition(":")
            fields[key.strip()] = val.strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if fields.get("kernel source sha256") != sha or "hbm bytes per launch" not in fields:
        return None
    return float(fields["hbm bytes per launch"])


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
    for mode, kw in (("batched_graph", dict(batched=True, graph=True)), ("plain", dict(batched=False))):
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


def serve_bench(args):
    """Serving: Poisson arrivals (20 / s) of regime-switching series with n
    log-uniform in [1e4, 5e5], m in {64, .., 1024}, l = m/2, K in 3..5."""
    import numpy as np
    import torch

    from paper_2401_13680_amd import api, synth

    reqs = synth.poisson_requests(num=args.requests, rate=20.0, seed=5)
    cells = sum((len(r.x) // r.m) * (r.m - r.l + 1) * (len(r.x) - r.l + 1) for r in reqs)
    # plain: one request after another with pst_snippets
    Ts = [torch.from_numpy(r.x).cuda() for r in reqs]
    api.snippets(Ts[0], reqs[0].m, reqs[0].l, reqs[0].K)
    torch.cuda.synchronize()
    plain_ms = []
    t0 = time.perf_counter()
    for r, T in zip(reqs, Ts):
        t1 = time.perf_counter()
        api.snippets(T, r.m, r.l, r.K)
        torch.cuda.synchronize()
        plain_ms.append((time.perf_counter() - t1) * 1e3)
    plain = time.perf_counter() - t0
    del Ts
    srv = api.Server(0, hbm_budget_bytes=96 << 30, max_slots=8)
    # saturation replay: everything submitted at once
    t0 = time.perf_counter()
    tk = [srv.submit(r.x, r.m, r.l, r.K) for r in reqs]
    srv.drain()
    sat = time.perf_counter() - t0
    for t in tk:
        srv.poll(t)
    # Poisson replay at the recorded arrival times
    t0 = time.perf_counter()
    tickets, lat = [], []
    for r in reqs:
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(r.x, r.m, r.l, r.K))
    srv.drain()
    span = time.perf_counter() - t0
    for t in tickets:
        lat.append(srv.poll(t)["latency_ms"])
    srv.close()
    # admission order under queueing (two slots, so requests wait): the same
    # Poisson replay in arrival order and shortest predicted first, the model
    # seeded with the plain pass's per-request times
    model = api.RuntimeModel(2)
    for r, ms in zip(reqs, plain_ms):
        model.observe(len(r.x), r.m, r.l, ms)
    model.fit()
    order = {}
    for name, pol in (("arrival", api.Server.ARRIVAL), ("shortest_predicted_first", api.Server.SHORTEST_PREDICTED)):
        srv = api.Server(0, hbm_budget_bytes=96 << 30, max_slots=2)
        srv.set_policy(pol, model if pol else None)
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            delay = r.arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(r.x, r.m, r.l, r.K))
        srv.drain()
        sp = time.perf_counter() - t0
        lt = [srv.poll(t)["latency_ms"] for t in tickets]
        srv.close()
        order[name] = dict(seconds=round(sp, 4), p50=round(float(np.percentile(lt, 50)), 2),
                           p99=round(float(np.percentile(lt, 99)), 2), mean=round(float(np.mean(lt)), 2))
    out = dict(metric="MPdist distance-matrix cells/sec on 1 MI355X; p50/p99 request latency",
               value=cells / sat, unit="cells/s", n_gpus=1, steps=1, warmup=1,
               ms_per_step=sat * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload="poisson20_regimes_serving", requests=len(reqs), cells=cells,
                           step="all requests submitted at once, served with overlap"),
               latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                               mean=float(np.mean(lat))),
               poisson_replay=dict(seconds=span, cells_per_s=cells / span),
               admission_order_two_slots=order,
               plain_one_request_at_a_time=dict(value=cells / plain, seconds=plain),
               served_over_plain=plain / sat)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="regimes5_n100000",
                    choices=["regimes5_n100000", "sweep", "serve", "multi", "schedule", "blocked"])
    ap.add_argument("--requests", type=int, default=40, help="serve: number of requests")
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
    if args.workload == "multi":
        return multi_bench(args)
    if args.workload == "schedule":
        return schedule_bench(args)
    if args.workload == "blocked":
        return blocked_bench(args)

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
                      frac=achieved / peak, traffic=measured_traffic(), kernel="k_profile",
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
