#!/usr/bin/env python
"""Range queries/s of the TUCKET stitch engine on one MI355X.

A step answers every query of the workload's query list in one batched
device launch (Recall, partial-hit trims and Stitch for each query, one
workgroup per query), with the node store already built and resident in
HBM.  Beside it the same queries run one per launch (the plain GPU path),
giving per-query latencies (p50/p99), and the FP64 CPU oracle is timed on a
bounded sample on the host cores.

Prints one JSON line (see the keys below).
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 (MFMA and packed vector)
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
HBM_TBPS = 8.0

# HBM bytes per step of a workload's stitch launches, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE per dispatch, summed over the step's
# launches) scaled by the counters of a reference copy of known size
# (`--copy-calibration`); keyed by (workload, precision) and valid only for
# the kernel sources (sha) and the launch tuning they were taken with.
TRAFFIC_BYTES_PER_STEP = {
    ("serving", "f32"): {"fetch": 12600994186, "write": 8685448800, "sha": "6e52f1886517641b",
                         "tuning": {"wide_threshold": 32, "wide_threads": 128, "persistent": 1, "graph": 1,
                                    "coarse": 1, "lds_n": 64, "basis_pct": 75, "rest_threads": 0,
                                    "wide_core": 0}},
}

# Launch tunings of the batched runs (tk_autotune's choices on MI355X for
# the serving workload's 4096-query list; `--autotune` searches again).
# The HBM counters above are taken under these.
TUNINGS = {
    ("serving", "f32"): {"wide_threshold": 32, "wide_threads": 128, "persistent": 1, "graph": 1, "coarse": 1,
                         "lds_n": 64, "basis_pct": 75, "rest_threads": 0, "wide_core": 0},
    ("serving", "bf16"): {"wide_threshold": 32, "wide_threads": 128, "persistent": 0, "graph": 1, "coarse": 1,
                          "lds_n": 48, "basis_pct": 75, "rest_threads": 0, "wide_core": 0},
}
KERNEL_SOURCES = ("tk_common.hpp", "tk_device.hpp", "tk_internal.hpp", "tk_kernels.hip", "tk_stitch.hpp",
                  "tk_stitch_inst.hip")


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_06647_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stitch_flops(p, D, rq, hits, node_ranks, sweeps, L):
    """Algorithmic FLOPs of one query (Alg. "stitch" on its hit set), counted
    from the shapes: per sweep, per hit the projections U^(m)T V~^(m), the
    temporal-mode TTM chain and the mode-n chains with their x_n V~ products;
    per query the Gram of each unfolding (smaller side) and the core update;
    once, the temporal factor rows and the partial-hit QRs."""
    if sweeps == 0:
        return 0.0
    r = list(rq)
    R = [math.prod(r[m] for m in range(p) if m != n) for n in range(p)]
    F = 0.0
    ksum = 0
    kbar = 0.0
    for h in hits:
        nr = node_ranks[h["level"]]
        k = nr[0]
        ksum += k
        kbar += k * (h["hi"] - h["lo"])
        f = sum(2.0 * D[m] * r[m] * nr[m] for m in range(1, p))
        f += sum(2.0 * k * R[0] * r[m] for m in range(1, p))
        for n in range(1, p):
            f += 2.0 * r[0] * k * R[0]
            f += sum(2.0 * r[0] * R[0] * r[m] for m in range(1, p) if m != n)
            f += 2.0 * D[n] * nr[n] * R[n]
        F += f
    Fq = 2.0 * min(ksum * ksum * R[0], R[0] * R[0] * ksum)
    Fq += sum(2.0 * min(D[n] * D[n] * R[n], R[n] * R[n] * D[n]) for n in range(1, p))
    Fq += 2.0 * r[p - 1] * D[p - 1] * R[p - 1]
    Ffin = 2.0 * L * r[0] * (kbar / max(L, 1))
    Ffin += sum(4.0 * (h["hi"] - h["lo"]) * node_ranks[h["level"]][0] ** 2 for h in hits if h["partial"])
    return sweeps * (F + Fq) + Ffin


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return 1


def serve_main(args):
    """Serving run: a short prefix of the stream is built, then slices are
    appended at a steady rate while range queries arrive as a Poisson
    process, each over a log-uniform length inside the horizon committed
    when it is submitted; the library's scheduler admits them into the
    running work as job slots and workspace free up.  Reports queries/s and
    p50/p99 latency (submission to completion, host clock), then the
    closed-loop append rate (a burst of appends submitted at once)."""
    # The serving engine drives five streams (the tree's, the appends', three
    # query classes); HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues
    # (4 by default), and an append commit sharing a queue with a class's
    # running launch waits for it.  --hw-queues (default 8) gives every
    # stream its own; it must be set before the runtime starts.
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import torch
    import synth
    from paper_2501_06647_amd import Tree
    from paper_2501_06647_amd.tucket import TK_BF16, TK_F32

    def say(msg):
        print("[serve] %s" % msg, file=sys.stderr, flush=True)

    say("GPU_MAX_HW_QUEUES=%s" % os.environ.get("GPU_MAX_HW_QUEUES"))

    wl = synth.get(args.workload)
    torch.cuda.set_device(0)
    rng = np.random.default_rng(wl.query_seed + 77)
    T0 = min(args.serve_prefix, wl.T)
    n_app = min(int(args.aps * args.serve_seconds), wl.T - T0 - args.burst_appends)
    t0 = time.perf_counter()
    Xd = _device_series(wl, T0 + n_app + args.burst_appends, torch.device("cuda:0"))
    say("generated %d slices in %.1f s" % (T0 + n_app + args.burst_appends, time.perf_counter() - t0))
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    tree.build(Xd[:T0])
    torch.cuda.synchronize()
    if not args.no_tune:
        ts, te = synth.queries(wl, T=T0, n=512)
        say("autotune: %s" % (tree.autotune(ts, te, reps=1, budget_s=30.0),))
    prec = TK_BF16 if args.serve_prec == "bf16" else TK_F32
    tree.set_query_prec(prec)
    # arrival schedule
    horizon = n_app / args.aps
    q_times = np.cumsum(rng.exponential(1.0 / args.qps, size=int(args.qps * horizon * 1.2) + 16))
    q_times = q_times[q_times < horizon]
    a_times = np.arange(n_app) / args.aps
    events = sorted([(t, 1, i) for i, t in enumerate(a_times)] + [(t, 0, i) for i, t in enumerate(q_times)])
    say("prefix %d slices, %d appends at %g/s, %d queries at %g/s over %.1f s, %s queries, FP32 merges"
        % (T0, n_app, args.aps, len(q_times), args.qps, horizon, args.serve_prec))
    srv = tree.serve(max_batch=args.serve_slots)
    ell = wl.leaf_len
    T = T0
    qtickets = []
    open_q = []
    lat = []
    lat_T = []       # horizon at each query's submission, in the order of lat
    q_T = {}
    atickets = []
    t_start = time.perf_counter()
    last_print = t_start
    for (tev, kind, i) in events:
        while True:
            now = time.perf_counter() - t_start
            if now >= tev:
                break
            if tev - now > 2e-4:
                time.sleep(min(tev - now - 1e-4, 1e-3))
        if kind == 1:
            atickets.append(srv.submit_append(Xd[T]))
            T += 1
        else:
            Tc = (T // ell) * ell
            if Tc < 1:
                continue
            L = int(min(Tc, max(1, round(math.exp(rng.uniform(0.0, math.log(Tc)))))))
            a = int(rng.integers(0, Tc - L + 1))
            tk = srv.submit_query(a, a + L)
            qtickets.append(tk)
            open_q.append(tk)
            q_T[tk] = T
        # take finished results so device memory stays bounded
        while open_q and srv.poll(open_q[0]):
            tk = open_q.pop(0)
            ts_, tl_, td_ = srv.times(tk)
            lat.append(td_ - ts_)
            lat_T.append(q_T.pop(tk))
            srv.release(tk)
        if time.perf_counter() - last_print > 5.0:
            last_print = time.perf_counter()
            say("t=%.1f s T=%d %s" % (last_print - t_start, T, srv.stats()))
    srv.sync()
    wall = time.perf_counter() - t_start
    for tk in open_q:
        ts_, tl_, td_ = srv.times(tk)
        lat.append(td_ - ts_)
        lat_T.append(q_T.pop(tk))
        srv.release(tk)
    a_lat = []
    for tk in atickets:
        ts_, tl_, td_ = srv.times(tk)
        a_lat.append(td_ - ts_)
        srv.release(tk)
    stats = srv.stats()
    # closed loop: a burst of appends submitted at once, committed as fast as the engine can
    t1 = time.perf_counter()
    for k in range(args.burst_appends):
        srv.submit_append(Xd[T + k])
    srv.sync()
    burst_s = time.perf_counter() - t1
    T += args.burst_appends
    srv.stop()
    lat_ms = np.array(lat) / 1000.0
    lat_T = np.array(lat_T)
    a_ms = np.array(a_lat) / 1000.0
    qps = len(qtickets) / wall
    # query latency against the horizon (quarters of the run's T range) and
    # append latency (submission to commit)
    edges = np.linspace(T0, T0 + n_app, 5)
    by_T = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (lat_T >= lo) & (lat_T < hi) if hi < edges[-1] else (lat_T >= lo)
        if m.any():
            by_T.append({"T": [int(lo), int(hi)], "queries": int(m.sum()),
                         "p50": float(np.percentile(lat_ms[m], 50)), "p99": float(np.percentile(lat_ms[m], 99))})
    out = {
        "metric": "serving: range queries/s with p50/p99 latency, appends interleaved",
        "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": len(qtickets), "warmup": 0,
        "ms_per_step": 1000.0 * wall / max(1, len(qtickets)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.serve_prec, "data": "synthetic",
        "config": {"workload": "%s: %s slices, T %d -> %d, node ranks %s, leaf %d; Poisson queries at %g/s "
                               "(log-uniform lengths in [1, T_c]), appends at %g/s, %s queries, FP32 merges, "
                               "%d job slots per class"
                               % (wl.name, "x".join(map(str, wl.dims)), T0, T, wl.node_ranks, wl.leaf_len,
                                  args.qps, args.aps, args.serve_prec, args.serve_slots)},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "latency_by_horizon_ms": by_T,
        "append_latency_ms": {"p50": float(np.percentile(a_ms, 50)), "p99": float(np.percentile(a_ms, 99)),
                              "max": float(a_ms.max())} if len(a_ms) else None,
        "appends_per_s": n_app / wall,
        "closed_loop_appends_per_s": args.burst_appends / burst_s,
        "server": stats,
    }
    print(json.dumps(out), flush=True)


def _rel_err(X, G, Us):
    """|X - G x_1 U1 ... x_p Up|_F / |X|_F in FP64 (the paper's error metric)."""
    Y = np.asarray(G, dtype=np.float64)
    for n, U in enumerate(Us):
        Y = np.moveaxis(np.tensordot(np.asarray(U, dtype=np.float64), Y, axes=(1, n)), 0, n)
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm((X - Y).ravel()) / max(1e-300, np.linalg.norm(X.ravel())))


def tradeoff_main(args):
    """The efficiency-accuracy comparison on the plain workload's
    regime-switched synthetic series: Alg. "recall" at theta 1/2, 7/10, 9/10
    and 1, and the fixed-block variant (blocks of about T / (2 ceil(log2 T))
    slices), each the whole query list as one prepared batch under one
    tuning; error of every sampled result against the raw data."""
    import torch
    import synth
    from paper_2501_06647_amd import Tree

    wl = synth.get(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X = synth.series(wl)
    Xd = torch.from_numpy(X.astype(np.float32)).to(dev)
    ts, te = synth.queries(wl)
    nq = len(ts)
    block = wl.T / (2 * math.ceil(math.log2(wl.T)))
    level = max(0, int(round(math.log2(block / wl.leaf_len))))
    sample = np.random.default_rng(3).choice(nq, size=min(nq, 256), replace=False)
    settings = [("recall", th) for th in ((1, 2), (7, 10), (9, 10), (1, 1))] + [("fixed", level)]
    tuning = None
    rows = []
    for kind, arg in settings:
        theta = arg if kind == "recall" else wl.theta
        tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, theta, wl.max_iter, wl.tol, capacity_T=wl.T)
        tree.build(Xd)
        if kind == "fixed":
            tree.set_query_recall(level)
        if tuning is None:
            tuning, _ = tree.autotune(ts, te, reps=2)
        else:
            tree.set_tuning(**tuning)
        b = tree.prepare_batch(ts, te)
        for _ in range(args.warmup):
            b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for _ in range(args.steps):
            b.run()
            kms.append(b.kernel_ms())
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / args.steps
        res = b.results()
        hits = [len(tree.hitset(int(ts[i]), int(te[i]))) for i in range(nq)]
        errs = []
        for i in sample:
            G = res[i].core.double().cpu().numpy()
            Us = [u.double().cpu().numpy() for u in res[i].factors]
            errs.append(_rel_err(X[int(ts[i]):int(te[i])], G, Us))
        row = {"hit_set": "recall theta %d/%d" % arg if kind == "recall" else
               "fixed blocks of %d slices (level %d)" % (wl.leaf_len << level, level),
               "queries_per_s": nq / (ms / 1000.0), "ms_per_step": ms, "kernel_ms": float(np.mean(kms)),
               "hits_mean": float(np.mean(hits)), "rel_err_mean": float(np.mean(errs)),
               "rel_err_p90": float(np.percentile(errs, 90)), "sweeps_mean": float(np.mean([r.sweeps for r in res]))}
        rows.append(row)
        print("[tradeoff] %s" % json.dumps(row), file=sys.stderr, flush=True)
        b.close()
        tree.close()
    # the naive baseline and accuracy reference: Tucker-ALS from scratch on each raw range
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = tree.raw_tucker(Xd, ts, te)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0)
    errs = []
    for i in sample:
        G = res[i].core.double().cpu().numpy()
        Us = [u.double().cpu().numpy() for u in res[i].factors]
        errs.append(_rel_err(X[int(ts[i]):int(te[i])], G, Us))
    row = {"hit_set": "none: Tucker-ALS from scratch on each raw range (tk_raw_tucker)",
           "queries_per_s": nq / (ms / 1000.0), "ms_per_step": ms, "hits_mean": 0.0,
           "rel_err_mean": float(np.mean(errs)), "rel_err_p90": float(np.percentile(errs, 90)),
           "sweeps_mean": float(np.mean([r.sweeps for r in res]))}
    rows.append(row)
    print("[tradeoff] %s" % json.dumps(row), file=sys.stderr, flush=True)
    tree.close()
    out = {"metric": "efficiency-accuracy tradeoff: range queries/s and relative error vs hit-set rule",
           "value": rows[1]["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s: %s x T=%d, leaf %d, ranks %s, %d queries, error sample %d"
                      % (wl.name, "x".join(str(d) for d in wl.dims), wl.T, wl.leaf_len, wl.node_ranks, nq,
                         len(sample)), "tuning": tuning},
           "settings": rows}
    print(json.dumps(out), flush=True)


def pscale_main(args):
    """Query latency and throughput against the number of modes on the
    paper's many-mode shapes (every slice 10^6 elements, rank 5 per mode,
    400 slices, leaf 1): p = 3 to 7; queries of 98, 192 and 384 slices
    from seeded random starts, one at a time (latency) and as one prepared
    batch (throughput)."""
    import torch
    import synth
    from synth.workloads import d5
    from paper_2501_06647_amd import Tree

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rows = []
    for p in [int(x) for x in args.pscale_p.split(",")]:
        wl = d5(p)
        tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
        gen_s, build_s = 0.0, 0.0
        for t0 in range(0, wl.T, 128):
            g0 = time.perf_counter()
            X = synth.series(wl, t0, min(wl.T, t0 + 128)).astype(np.float32)
            Xd = torch.from_numpy(X).to(dev)
            gen_s += time.perf_counter() - g0
            torch.cuda.synchronize()
            b0 = time.perf_counter()
            tree.build(Xd)
            torch.cuda.synchronize()
            build_s += time.perf_counter() - b0
            print("[pscale] p=%d: slices [%d, %d) generated and appended" % (p, t0, min(wl.T, t0 + 128)),
                  file=sys.stderr, flush=True)
            del X, Xd
        print("[pscale] p=%d %s: data %.1f s, build %.2f s" % (p, "x".join(str(d) for d in wl.dims), gen_s, build_s),
              file=sys.stderr, flush=True)
        rng = np.random.default_rng(40 + p)
        tts = rng.integers(0, wl.T - 192 + 1, size=64).astype(np.int64)
        if args.pscale_tuning:
            tuning = json.loads(args.pscale_tuning)
            tree.set_tuning(**tuning)
        elif p in [int(x) for x in args.pscale_tune_p.split(",") if x]:
            tuning, _ = tree.autotune(tts, tts + 192, reps=1)
        elif rows:
            # the grid search costs ~150 batches: at many modes reuse the
            # tuning chosen for the previous p
            tuning = rows[-1]["tuning"]
            tree.set_tuning(**tuning)
        else:
            tuning = tree.tuning()
        print("[pscale] p=%d tuning: %s" % (p, tuning), file=sys.stderr, flush=True)
        for L in (98, 192, 384):
            ts = rng.integers(0, wl.T - L + 1, size=64).astype(np.int64)
            te = ts + L
            lat = []
            for a, c in zip(ts[:16].tolist(), te[:16].tolist()):
                t1 = time.perf_counter()
                tree.query(a, c)
                lat.append(time.perf_counter() - t1)
            print("[pscale] p=%d L=%d: 16 single queries, p50 %.2f ms" % (p, L, 1000.0 * float(np.median(lat))),
                  file=sys.stderr, flush=True)
            b = tree.prepare_batch(ts, te)
            for _ in range(args.warmup):
                b.run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                b.run()
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - t1) / args.steps
            res = b.results()
            prof = [b.profile(i) for i in range(len(ts))]
            phases = {k: round(float(np.mean([pr[k] for pr in prof])), 1) for k in tree.PHASES}
            hits = [len(tree.hitset(int(a), int(c))) for a, c in zip(ts, te)]
            row = {"p": p, "dims": list(wl.dims), "L": L, "tuning": tuning, "build_s": build_s,
                   "latency_p50_ms": 1000.0 * float(np.median(lat)),
                   "latency_p99_ms": 1000.0 * float(np.percentile(lat, 99)), "batch_queries": len(ts),
                   "batch_queries_per_s": len(ts) / (ms / 1000.0), "hits_mean": float(np.mean(hits)),
                   "sweeps_mean": float(np.mean([r.sweeps for r in res])), "phase_mean_us": phases}
            rows.append(row)
            print("[pscale] %s" % json.dumps(row), file=sys.stderr, flush=True)
            b.close()
        tree.close()
    out = {"metric": "range-query latency vs number of modes (many-mode shapes, rank 5)",
           "value": rows[-1]["latency_p50_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "slices of 10^6 elements (100^3, 100^2 x 10^2, 100 x 10^4, 10^6), 400 slices, leaf 1, "
                                  "rank 5, queries of 98/192/384 slices"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def copy_calibration_main(args):
    """A device-to-device copy of a known size (PyTorch's copy kernel), for
    converting rocprofv3's FETCH_SIZE / WRITE_SIZE counters into bytes: each
    copy reads and writes args.copy_mib MiB."""
    import torch
    n = args.copy_mib * (1 << 20) // 4
    src = torch.randn(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied 3 x %d MiB" % args.copy_mib, flush=True)


def cpu_info():
    """Host cores and CPU model (for the oracle baseline's record)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def raw_main(args):
    """Tucker-ALS from scratch on long raw ranges of the serving workload's
    series (128 x 128 slices, ranks 16): the many-workgroup streaming
    decomposition (tk_raw_tucker_stream) at several lengths, and the
    one-workgroup-per-range kernel (tk_raw_tucker) on the shortest.  Each
    pass reads the range once ((p - 1) HOSVD passes, then p per sweep), so
    the effective read bandwidth is passes x bytes / time, against HBM's."""
    import torch
    import synth
    from paper_2501_06647_amd import Tree

    wl = synth.get(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lens = [int(x) for x in args.raw_lengths.split(",")]
    T = max(lens)
    t0 = time.perf_counter()
    Xd = _device_series(wl, T, dev)
    print("[raw] generated %d slices in %.1f s" % (T, time.perf_counter() - t0), file=sys.stderr, flush=True)
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    slice_bytes = int(np.prod(wl.dims)) * 4
    p = 1 + len(wl.dims)
    rows = []
    for L in lens:
        r = tree.raw_tucker_stream(Xd, 0, L)  # warm-up (buffers)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t1 = time.perf_counter()
            r = tree.raw_tucker_stream(Xd, 0, L)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        sec = float(np.median(ts))
        passes = (p - 1) + p * r.sweeps
        gbs = passes * L * slice_bytes / sec / 1e9
        row = {"L": L, "ms": 1000 * sec, "sweeps": r.sweeps, "passes": passes, "read_GB_per_s": gbs,
               "hbm_frac": gbs / (HBM_TBPS * 1000), "err_model": r.err_model}
        rows.append(row)
        print("[raw] streaming %s" % json.dumps(row), file=sys.stderr, flush=True)
    L = min(lens)
    t1 = time.perf_counter()
    one = tree.raw_tucker(Xd, np.array([0]), np.array([L]))[0]
    torch.cuda.synchronize()
    one_ms = 1000 * (time.perf_counter() - t1)
    print("[raw] one workgroup per range, L=%d: %.1f ms (%d sweeps)" % (L, one_ms, one.sweeps), file=sys.stderr,
          flush=True)
    tree.close()
    out = {"metric": "Tucker-ALS from scratch on a raw range (streaming, many workgroups)", "unit": "ms",
           "config": {"workload": "%s: %s slices, ranks %s, <=%d sweeps, tol %g"
                                  % (wl.name, "x".join(map(str, wl.dims)), wl.node_ranks, wl.max_iter, wl.tol)},
           "streaming": rows, "one_workgroup": {"L": L, "ms": one_ms, "sweeps": one.sweeps}}
    print(json.dumps(out), flush=True)


def _device_series(wl, T, dev, chunk=4096):
    """The workload's first T slices as one FP32 device tensor, generated in
    chunks (host memory stays at one chunk)."""
    import torch
    import synth
    Xd = torch.empty((T,) + tuple(wl.dims), dtype=torch.float32, device=dev)
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        Xd[t0:t1].copy_(torch.from_numpy(synth.series(wl, t0, t1).astype(np.float32)))
    return Xd


def _time_batch(batch, steps, warmup):
    """Warm-up runs, then `steps` graph replays bracketed by device
    synchronisation; returns (ms per step on the host clock, mean kernel ms
    from HIP events on the tree's stream)."""
    import torch
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run()
        kms.append(batch.kernel_ms())
    torch.cuda.synchronize()
    return 1000.0 * (time.perf_counter() - t0) / steps, float(np.mean(kms))


def _device_latency(batch, n):
    """Per-query completion latency of one batched step from the kernel's own
    clock (100 MHz): each query's end time minus the step's first start (all
    queries are submitted together), and each query's execution time."""
    prof = [batch.profile(i) for i in range(n)]
    t_s = np.array([pr["start_us"] for pr in prof])
    t_e = np.array([pr["end_us"] for pr in prof])
    done = t_e - t_s.min()
    run = t_e - t_s
    return prof, {"completion_p50_ms": float(np.percentile(done, 50)) / 1000.0,
                  "completion_p99_ms": float(np.percentile(done, 99)) / 1000.0,
                  "exec_p50_ms": float(np.percentile(run, 50)) / 1000.0,
                  "exec_p99_ms": float(np.percentile(run, 99)) / 1000.0,
                  "makespan_ms": float(t_e.max() - t_s.min()) / 1000.0,
                  "mean_concurrency": float(run.sum() / max(1e-9, t_e.max() - t_s.min()))}


def _flops(tree, wl, ts, te, results):
    D = [0] + list(wl.dims)
    node_ranks = {k: tree.node_ranks(k) for k in range(40) if (wl.leaf_len << k) <= wl.T}
    flops = 0.0
    hits_n = []
    for i in range(len(ts)):
        hits = tree.hitset(int(ts[i]), int(te[i]))
        r = results[i]
        flops += stitch_flops(tree.p, D, r.ranks, hits, node_ranks, r.sweeps, int(te[i] - ts[i]))
        hits_n.append(len(hits))
    return flops, hits_n


def _accuracy(tree, wl, prefix, nq, precs, say):
    """Error of the device results against the FP64 oracle on a fixed sample
    of queries inside the first `prefix` slices: the oracle builds its own
    tree over that prefix from the raw data (subtrees in worker processes)
    and answers the same queries; |e_gpu / e_oracle - 1| per precision, e
    the relative error against the raw data.  Also times the oracle's
    queries (the CPU baseline)."""
    import synth
    from paper_2501_06647_amd.tucket import TK_F32
    from oracle import pool
    from oracle.evaluate import relative_error
    from threadpoolctl import threadpool_limits
    ts, te = synth.queries(wl, T=prefix, n=nq, seed_offset=17)
    out = {"sample": "%d queries of the workload's length distribution inside [0, %d)" % (nq, prefix)}
    dev = {}
    for name, prec in precs:
        tree.set_query_prec(prec)
        b = tree.prepare_batch(ts, te)
        b.run()
        dev[name] = [(r.core.double().cpu().numpy(), [u.double().cpu().numpy() for u in r.factors])
                     for r in b.results()]
        b.close()
    tree.set_query_prec(TK_F32)
    t0 = time.perf_counter()
    orc = pool.lazy_tree(wl, prefix)
    level = pool.pool_level(wl)
    pool.fill(orc, wl, level, range(prefix // (wl.leaf_len << level)))
    for v in orc.complete_nodes():
        orc.ensure(v)
    build_s = time.perf_counter() - t0
    say("oracle prefix of %d slices built in %.1f s (%d worker processes)" % (prefix, build_s, pool.workers()))
    X = synth.series(wl, 0, prefix)
    deltas = {name: [] for name in dev}
    errs = {name: [] for name in dev}
    q_s = 0.0
    blas = 1
    with threadpool_limits(1):
        for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
            t1 = time.perf_counter()
            Go, Uo, _ = orc.query(a, c)
            q_s += time.perf_counter() - t1
            e_o = relative_error(X[a:c], Go, Uo)
            for name in dev:
                G, U = dev[name][i]
                e_g = relative_error(X[a:c], G, U)
                deltas[name].append(abs(e_g / e_o - 1.0) if e_o > 0 else e_g)
                errs[name].append(e_g)
    for name in dev:
        out[name] = {"max_err_ratio_delta": float(max(deltas[name])),
                     "p99_err_ratio_delta": float(np.percentile(deltas[name], 99)),
                     "median_rel_err": float(np.median(errs[name])),
                     "gate": 1e-5 if name == "f32" else 1e-2}
    cpu = {"value": nq / q_s, "unit": "queries/s", "cores": blas, "kind": "oracle",
           "sample": "FP64 NumPy oracle (one BLAS thread): Recall, QR trims and Stitch with Z^(1) materialised "
                     "for the %d accuracy queries inside [0, %d) (%.1f s of query time); its tree over that "
                     "prefix built from the raw slices by %d worker processes in %.1f s (%.1f slices/s)"
                     % (nq, prefix, q_s, pool.workers(), build_s, prefix / build_s)}
    cpu.update(cpu_info())
    return out, cpu


def batched_main(args):
    """The headline: a step answers the workload's whole query list as one
    prepared batch (HIP graph replay; Recall, trims and Stitch of every query
    on the device), node store built and resident in HBM; FP32 and BF16
    contractions; beside it the plain one-query-per-launch FP32 path,
    streamed appends, accuracy against the oracle and the oracle's speed."""
    import torch
    import synth
    from paper_2501_06647_amd import Tree
    from paper_2501_06647_amd.tucket import TK_BF16, TK_F32

    def say(msg):
        print("[bench] %s" % msg, file=sys.stderr, flush=True)

    wl = synth.get(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    Xd = _device_series(wl, wl.T, dev)
    say("generated %s: %d slices of %s in %.1f s" % (wl.name, wl.T, "x".join(map(str, wl.dims)),
                                                    time.perf_counter() - t0))
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree.build(Xd)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    say("built the tree from device-resident slices in %.3f s (%.0f slices/s)" % (build_s, wl.T / build_s))

    # streamed appends: one slice per tk_append call, as a stream arrives
    app = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    n_app = min(wl.T, args.append_slices)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < n_app:
        app.append(Xd[done])
        done += 1
        if time.perf_counter() - t0 > args.append_seconds:
            break
    torch.cuda.synchronize()
    app_s = time.perf_counter() - t0
    appends = {"streamed_per_s": done / app_s, "streamed_slices": done,
               "bulk_build_per_s": wl.T / build_s, "merges_total": app.stats()["merges_total"]}
    app.close()
    say("streamed appends: %d slices one per call, %.0f slices/s" % (done, done / app_s))

    ts, te = synth.queries(wl)
    nq = len(ts)
    precs = [("f32", TK_F32)] + ([] if args.no_bf16 else [("bf16", TK_BF16)])
    runs = {}
    for name, prec in precs:
        tree.set_query_prec(prec)
        if args.tuning:
            tree.set_tuning(**json.loads(args.tuning))
        elif args.autotune or (wl.name, name) not in TUNINGS:
            t0 = time.perf_counter()
            tuning, tune_ms = tree.autotune(ts, te, reps=2)
            say("%s autotune: %s (%.3f ms per batch) in %.1f s" % (name, tuning, tune_ms, time.perf_counter() - t0))
        else:
            tree.set_tuning(**TUNINGS[(wl.name, name)])
        batch = tree.prepare_batch(ts, te)
        ms, kms = _time_batch(batch, args.steps, args.warmup)
        batch.run()
        prof, lat = _device_latency(batch, nq)
        results = batch.results()
        flops, hits_n = _flops(tree, wl, ts, te, results)
        peak = PEAK_FP32_TFLOPS if name == "f32" else PEAK_BF16_TFLOPS
        achieved = flops / (kms / 1000.0) / 1e12
        phases = {k: float(np.mean([pr[k] for pr in prof])) for k in tree.PHASES}
        eig = {k: float(np.mean([pr[k] for pr in prof])) for k in tree.COUNTERS[:4] + tree.COUNTERS[6:]}
        runs[name] = {"queries_per_s": nq / (ms / 1000.0), "ms_per_step": ms, "kernel_ms": kms,
                      "tuning": tree.tuning(), "latency": lat,
                      "sweeps_mean": float(np.mean([r.sweeps for r in results])),
                      "hits_mean": float(np.mean(hits_n)),
                      "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                                   "frac": achieved / peak, "gflop_per_launch": flops / 1e9},
                      "phase_mean_us": phases, "eig_mean": eig}
        say("%s batched: %.3f ms/step (kernel %.3f ms), %.0f queries/s, %.2f TFLOP/s (%.2f%% of peak); "
            "latency %s" % (name, ms, kms, nq / (ms / 1000.0), achieved, 100.0 * achieved / peak,
                             json.dumps({k: round(v, 3) for k, v in lat.items()})))
        say("%s phase mean us: %s; eigensolver: %s" % (name, json.dumps({k: round(v, 1) for k, v in phases.items()}),
                                                     json.dumps({k: round(v, 1) for k, v in eig.items()})))
        runs[name]["_batch"] = batch
    tree.set_query_prec(TK_F32)

    # the plain GPU path: one FP32 query per launch, no graph
    plain = None
    if not args.no_plain:
        b32 = runs["f32"]["_batch"]
        idx = list(range(0, nq, max(1, nq // args.plain_queries)))[:args.plain_queries]
        lat = []
        for i in idx:
            t1 = time.perf_counter()
            b32.run_one(i)
            lat.append(time.perf_counter() - t1)
        lat = np.array(lat)
        plain = {"queries_per_s": float(len(idx) / lat.sum()), "p50_ms": float(1000 * np.percentile(lat, 50)),
                 "p99_ms": float(1000 * np.percentile(lat, 99)), "launches": len(idx),
                 "sample": "every %d-th query of the list (host clock per call, launch to completion)"
                           % max(1, nq // args.plain_queries)}
        say("plain FP32, one query per launch: %.1f queries/s, p50 %.3f ms, p99 %.3f ms over %d queries"
            % (plain["queries_per_s"], plain["p50_ms"], plain["p99_ms"], len(idx)))
    for r in runs.values():
        r.pop("_batch").close()

    accuracy, cpu = None, None
    if not args.no_cpu:
        accuracy, cpu = _accuracy(tree, wl, min(args.acc_prefix, wl.T), args.acc_queries, precs, say)
        say("accuracy vs oracle: %s" % json.dumps(accuracy))

    head = args.headline if args.headline in runs else "f32"
    h = runs[head]
    traffic = None
    tb = TRAFFIC_BYTES_PER_STEP.get((wl.name, head))
    if tb and kernel_sha() == tb["sha"] and all(h["tuning"].get(k) == v for k, v in tb["tuning"].items()):
        traffic = tb["fetch"] + tb["write"]
    roof = dict(h["roofline"])
    roof.update({"traffic": traffic, "kernel": "stitch_kernel (all LDS-bin launches of the step)",
                 "kernel_ms": h["kernel_ms"]})
    out = {
        "metric": "range queries/sec at fixed rel. error; p50/p99 query latency vs plain GPU path",
        "value": h["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "%s: %s x T=%d FP32 series (%s), true rank %s, noise %.2f, leaf %d, node ranks %s; "
                               "%d queries per step (%s lengths), theta %d/%d, <=%d sweeps, tol %g; the whole "
                               "list as one prepared batch (HIP graph), node store resident in HBM"
                               % (wl.name, "x".join(map(str, wl.dims)), wl.T,
                                  "drifting factors" if wl.drift else "regime-switched" if wl.regime else "stationary",
                                  wl.true_ranks, wl.noise, wl.leaf_len, wl.node_ranks, nq, wl.query_kind,
                                  wl.theta[0], wl.theta[1], wl.max_iter, wl.tol),
                   "queries_per_step": nq, "headline_precision": head},
        "latency_ms": {"batched_completion_p50": h["latency"]["completion_p50_ms"],
                       "batched_completion_p99": h["latency"]["completion_p99_ms"],
                       "batched_exec_p50": h["latency"]["exec_p50_ms"],
                       "batched_exec_p99": h["latency"]["exec_p99_ms"],
                       "plain_p50": plain["p50_ms"] if plain else None,
                       "plain_p99": plain["p99_ms"] if plain else None},
        "precisions": runs,
        "plain_gpu_path": plain,
        "speedup_vs_plain": {k: r["queries_per_s"] / plain["queries_per_s"] for k, r in runs.items()} if plain else None,
        "appends": appends,
        "roofline": roof,
        "accuracy_vs_oracle": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    help="workload name (default: serving; plain for --tradeoff, whose from-scratch "
                         "baseline decomposes every raw range in one workgroup)")
    ap.add_argument("--headline", default="f32", help="precision of the headline value: f32 or bf16")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--append-slices", type=int, default=4096, help="streamed appends timed (one slice per call)")
    ap.add_argument("--append-seconds", type=float, default=10.0)
    ap.add_argument("--plain-queries", type=int, default=512, help="queries timed on the plain path")
    ap.add_argument("--acc-prefix", type=int, default=4096, help="oracle tree horizon for the accuracy sample")
    ap.add_argument("--acc-queries", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuning", default=None, help="JSON tuning for the batched runs")
    ap.add_argument("--autotune", action="store_true",
                    help="search the batched runs' tuning (tk_autotune) instead of the stored one")
    ap.add_argument("--serve", action="store_true", help="serving run instead of the batched benchmark")
    ap.add_argument("--qps", type=float, default=2000.0)
    ap.add_argument("--aps", type=float, default=1000.0)
    ap.add_argument("--serve-seconds", type=float, default=63.0,
                    help="serving run length: at 1000 appends/s from 256 slices the horizon reaches 63256")
    ap.add_argument("--serve-prefix", type=int, default=256)
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="GPU_MAX_HW_QUEUES for the serving run (0: leave the environment's)")
    ap.add_argument("--serve-prec", default="f32", help="query arithmetic while serving: f32 or bf16")
    ap.add_argument("--serve-slots", type=int, default=256, help="job slots (concurrent queries) per class")
    ap.add_argument("--burst-appends", type=int, default=2048, help="closed-loop appends after the serving run")
    ap.add_argument("--pscale", action="store_true", help="latency against the number of modes (p = 3..7)")
    ap.add_argument("--pscale-p", default="3,4,5,6,7", help="numbers of modes for --pscale")
    ap.add_argument("--pscale-tune-p", default="3,4,5,6",
                    help="numbers of modes autotuned in --pscale (the others reuse the previous tuning)")
    ap.add_argument("--pscale-tuning", default=None, help="JSON tuning for every p of --pscale")
    ap.add_argument("--raw", action="store_true",
                    help="Tucker-ALS from scratch on long raw ranges (streaming, many workgroups)")
    ap.add_argument("--raw-lengths", default="4096,16384,65536", help="range lengths for --raw")
    ap.add_argument("--tradeoff", action="store_true",
                    help="theta sweep and fixed-block variant: throughput and error per hit-set rule")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a device copy of --copy-mib MiB (HBM counter calibration under rocprofv3)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration_main(args)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(queries are independent: several GPUs would each hold a copy of the node store "
              "and take a share of the queries)", file=sys.stderr)
        sys.exit(2)
    if args.tradeoff:
        args.workload = args.workload or "plain"
        return tradeoff_main(args)
    args.workload = args.workload or "serving"
    if args.serve:
        return serve_main(args)
    if args.raw:
        return raw_main(args)
    if args.pscale:
        return pscale_main(args)
    return batched_main(args)


if __name__ == "__main__":
    main()
