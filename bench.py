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
HBM_TBPS = 8.0

# HBM bytes per step of the plain workload's stitch launches, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE per dispatch, summed over the
# step's launches) scaled by the counters of a 1 GiB reference copy (FETCH
# reads half the bytes moved, WRITE all of them); valid only for the kernel
# sources they were taken with.
TRAFFIC_KERNEL_SHA = "e1f56f3943b2a678"
TRAFFIC_BYTES_PER_STEP = {"plain": {"fetch": 1068.3e6, "write": 950.4e6,
                                    "tuning": {"wide_threshold": 32, "wide_threads": 128, "persistent": 0, "graph": 1,
                                               "coarse": 1, "lds_n": 64, "basis_pct": 75, "rest_threads": 256}}}
KERNEL_SOURCES = ("tk_common.hpp", "tk_device.hpp", "tk_internal.hpp", "tk_kernels.hip")


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
    """Serving run: a prefix of the stream is built, then slices are appended
    at a steady rate while range queries arrive as a Poisson process, each
    over a log-uniform length inside the horizon committed so far; the
    library's scheduler admits and batches them.  Reports queries/s and
    p50/p99 latency (submission to completion, host clock)."""
    import torch
    import synth
    from paper_2501_06647_amd import Tree

    wl = synth.get(args.workload)
    torch.cuda.set_device(0)
    rng = np.random.default_rng(wl.query_seed + 77)
    T0 = min(args.serve_prefix, wl.T)
    n_app = min(int(args.aps * args.serve_seconds), wl.T - T0)
    X = synth.series(wl, 0, T0 + n_app).astype(np.float32)
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    tree.build(X[:T0])
    torch.cuda.synchronize()
    if not args.no_tune:
        ts, te = synth.queries(wl, T=T0, n=512)
        print("[serve] autotune: %s" % (tree.autotune(ts, te, reps=1),), file=sys.stderr, flush=True)
    # arrival schedule
    horizon = n_app / args.aps
    q_times = np.cumsum(rng.exponential(1.0 / args.qps, size=int(args.qps * horizon * 1.2) + 16))
    q_times = q_times[q_times < horizon]
    a_times = np.arange(n_app) / args.aps
    events = sorted([(t, 1, i) for i, t in enumerate(a_times)] + [(t, 0, i) for i, t in enumerate(q_times)])
    print("[serve] prefix %d slices, %d appends at %g/s, %d queries at %g/s over %.1f s"
          % (T0, n_app, args.aps, len(q_times), args.qps, horizon), file=sys.stderr, flush=True)
    srv = tree.serve()
    ell = wl.leaf_len
    T = T0
    qtickets = []
    open_q = []
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
            srv.submit_append(X[T])
            T += 1
        else:
            Tc = (T // ell) * ell
            L = int(min(Tc, max(1, round(math.exp(rng.uniform(0.0, math.log(Tc)))))))
            a = int(rng.integers(0, Tc - L + 1))
            tk = srv.submit_query(a, a + L)
            qtickets.append(tk)
            open_q.append(tk)
        # release finished outputs so device memory stays bounded
        while open_q and srv.poll(open_q[0]):
            srv.release(open_q.pop(0))
        if time.perf_counter() - last_print > 5.0:
            last_print = time.perf_counter()
            print("[serve] t=%.1f s T=%d %s" % (last_print - t_start, T, srv.stats()), file=sys.stderr, flush=True)
    srv.sync()
    wall = time.perf_counter() - t_start
    stats = srv.stats()
    lat = np.array([srv.times(tk) for tk in qtickets])
    srv.stop()
    lat_ms = (lat[:, 2] - lat[:, 0]) / 1000.0
    qps = len(qtickets) / wall
    out = {
        "metric": "serving: range queries/s with p50/p99 latency, appends interleaved",
        "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": len(qtickets), "warmup": 0,
        "ms_per_step": 1000.0 * wall / max(1, len(qtickets)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: %s slices, T %d -> %d, node ranks %s, leaf %d; Poisson queries at %g/s "
                               "(log-uniform lengths in [1, T_c]), appends at %g/s"
                               % (wl.name, "x".join(map(str, wl.dims)), T0, T, wl.node_ranks, wl.leaf_len,
                                  args.qps, args.aps)},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "appends_per_s": n_app / wall,
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
    400 slices, leaf 1): p = 4 to 7; queries of 98, 192 and 384 slices
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
            row = {"p": p, "dims": list(wl.dims), "L": L, "tuning": tuning, "latency_p50_ms": 1000.0 * float(np.median(lat)),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuning", default=None, help="JSON tuning to use instead of autotuning")
    ap.add_argument("--serve", action="store_true", help="serving run instead of the batched benchmark")
    ap.add_argument("--qps", type=float, default=2000.0)
    ap.add_argument("--aps", type=float, default=1000.0)
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-prefix", type=int, default=4096)
    ap.add_argument("--pscale", action="store_true", help="latency against the number of modes (p = 4..7)")
    ap.add_argument("--pscale-p", default="4,5,6,7", help="numbers of modes for --pscale")
    ap.add_argument("--pscale-tune-p", default="4,5,6",
                    help="numbers of modes autotuned in --pscale (the others reuse the previous tuning)")
    ap.add_argument("--pscale-tuning", default=None, help="JSON tuning for every p of --pscale")
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
              "(queries are independent; see DESIGN.md on sharding)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        if args.workload == "plain":
            args.workload = "serving"
        return serve_main(args)
    if args.tradeoff:
        return tradeoff_main(args)
    if args.pscale:
        return pscale_main(args)

    import torch
    import synth
    from paper_2501_06647_amd import Tree

    wl = synth.get(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X = synth.series(wl)
    Xd = torch.from_numpy(X.astype(np.float32)).to(dev)
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=wl.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree.build(Xd)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    print("[bench] built %s tree: %d slices in %.3f s" % (wl.name, wl.T, build_s), file=sys.stderr, flush=True)

    ts, te = synth.queries(wl)
    nq = len(ts)
    tuning, tune_ms = None, None
    if args.tuning:
        tree.set_tuning(**json.loads(args.tuning))
    elif not args.no_tune:
        t0 = time.perf_counter()
        tuning, tune_ms = tree.autotune(ts, te, reps=2)
        print("[bench] autotune: %s (%.3f ms per batch) in %.1f s" % (tuning, tune_ms, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    tuning = tree.tuning()
    batch = tree.prepare_batch(ts, te)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
        kms.append(batch.kernel_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    qps = nq * args.steps / wall
    print("[bench] batched (graph): %.3f ms/step, kernel %.3f ms" % (ms_per_step, float(np.mean(kms))),
          file=sys.stderr, flush=True)
    # the same queries through tk_query_batch (host Recall and planning every call)
    sync_steps = max(1, min(3, args.steps))
    t1 = time.perf_counter()
    for _ in range(sync_steps):
        batch.run_sync()
    torch.cuda.synchronize()
    sync_ms = 1000.0 * (time.perf_counter() - t1) / sync_steps
    print("[bench] batched (tk_query_batch): %.3f ms/step" % sync_ms, file=sys.stderr, flush=True)
    batch.run()

    results = batch.results()
    D = [0] + list(wl.dims)
    node_ranks = {k: tree.node_ranks(k) for k in range(40) if (wl.leaf_len << k) <= wl.T}
    flops = 0.0
    sweeps = []
    hit_counts = []
    for i in range(nq):
        hits = tree.hitset(int(ts[i]), int(te[i]))
        res = results[i]
        flops += stitch_flops(tree.p, D, res.ranks, hits, node_ranks, res.sweeps, int(te[i] - ts[i]))
        sweeps.append(res.sweeps)
        hit_counts.append(len(hits))
    kernel_s = float(np.mean(kms)) / 1000.0
    achieved = flops / kernel_s / 1e12
    prof = [batch.profile(i) for i in range(nq)]
    phase_mean = {k: float(np.mean([pr[k] for pr in prof])) for k in tree.PHASES}
    tot = np.array([sum(pr[k] for k in tree.PHASES) for pr in prof])
    counters = {k: float(np.mean([pr[k] for pr in prof])) for k in tree.COUNTERS[:4] + tree.COUNTERS[6:]}
    t_s = np.array([pr["start_us"] for pr in prof])
    t_e = np.array([pr["end_us"] for pr in prof])
    t_base = t_s.min()
    timeline = {"makespan_us": float(t_e.max() - t_base),
                "start_offset_us_p50": float(np.median(t_s - t_base)),
                "start_offset_us_max": float((t_s - t_base).max()),
                "mean_concurrency": float((t_e - t_s).sum() / max(1e-9, t_e.max() - t_base))}
    print("[bench] device timeline: %s" % json.dumps({k: round(v, 1) for k, v in timeline.items()}),
          file=sys.stderr, flush=True)
    print("[bench] eigensolver per query: %s" % json.dumps({k: round(v, 1) for k, v in counters.items()}),
          file=sys.stderr, flush=True)
    slow = int(np.argmax(tot))
    print("[bench] phase mean us: %s" % json.dumps({k: round(v, 1) for k, v in phase_mean.items()}),
          file=sys.stderr, flush=True)
    print("[bench] per-query device us: mean %.1f p50 %.1f max %.1f (query %d, %d hits, L=%d)"
          % (tot.mean(), np.median(tot), tot.max(), slow, hit_counts[slow], int(te[slow] - ts[slow])),
          file=sys.stderr, flush=True)
    slowest = {"query": slow, "hits": hit_counts[slow], "L": int(te[slow] - ts[slow]),
               "sweeps": int(sweeps[slow]), "ranks": [int(r) for r in results[slow].ranks],
               "phases_us": {k: float(prof[slow][k]) for k in tree.PHASES},
               "eig": {k: float(prof[slow][k]) for k in tree.COUNTERS[:4] + tree.COUNTERS[7:]}}
    print("[bench] slowest query: %s" % json.dumps(slowest), file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        lat = []
        for i in range(nq):
            t1 = time.perf_counter()
            batch.run_one(i)
            lat.append(time.perf_counter() - t1)
        lat = np.array(lat)
        plain = {"queries_per_s": float(nq / lat.sum()), "p50_ms": float(1000 * np.percentile(lat, 50)),
                 "p99_ms": float(1000 * np.percentile(lat, 99)), "launches": nq}
        print("[bench] plain: %.1f q/s p50 %.3f ms p99 %.3f ms" % (plain["queries_per_s"], plain["p50_ms"],
                                                                 plain["p99_ms"]), file=sys.stderr, flush=True)

    cpu = None
    accuracy = None
    if not args.no_cpu:
        from oracle.evaluate import relative_error
        from oracle.tree import StreamSegmentTree
        t0 = time.perf_counter()
        orc = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol)
        for b in range(wl.T // wl.leaf_len):
            orc.append(X[b * wl.leaf_len:(b + 1) * wl.leaf_len])
        orc_build_s = time.perf_counter() - t0
        done, qt, deltas, errs = 0, 0.0, [], []
        while done < nq and qt < args.cpu_seconds:
            a, b = int(ts[done]), int(te[done])
            t1 = time.perf_counter()
            Go, Uo, _ = orc.query(a, b)
            qt += time.perf_counter() - t1
            r = results[done]
            e_g = relative_error(X[a:b], r.core.double().cpu().numpy(), [u.double().cpu().numpy() for u in r.factors])
            e_o = relative_error(X[a:b], Go, Uo)
            deltas.append(abs(e_g / e_o - 1.0) if e_o > 0 else e_g)
            errs.append(e_g)
            done += 1
        cpu = {"value": done / qt, "unit": "queries/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "FP64 NumPy oracle: tree built over all %d slices (%.1f s, %.0f slices/s), then "
                         "queries 0..%d of the same query list (Recall, QR trims, Stitch with Z^(1) "
                         "materialised), %.1f s of query time" % (wl.T, orc_build_s, wl.T / orc_build_s,
                                                                 done - 1, qt)}
        accuracy = {"n_checked": done, "max_err_ratio_delta": float(max(deltas)),
                    "median_rel_err": float(np.median(errs)), "gate": 1e-5}

    traffic, traffic_detail = None, None
    tb = TRAFFIC_BYTES_PER_STEP.get(wl.name)
    if tb and kernel_sha() == TRAFFIC_KERNEL_SHA:
        traffic = tb["fetch"] + tb["write"]
        traffic_detail = {"fetch_bytes": tb["fetch"], "write_bytes": tb["write"],
                          "GBps_at_kernel_ms": traffic / kernel_s / 1e9,
                          "measured_with_tuning": tb["tuning"],
                          "source": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch, copy-calibrated"}
    out = {
        "metric": "range queries/sec at fixed rel. error; p50/p99 query latency vs plain GPU path",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s x T=%d FP32 series, true rank %s, noise %.2f, leaf %d, node ranks %s, "
                               "%d queries (%s lengths), theta %d/%d, <=%d sweeps, tol %g"
                               % (wl.name, "x".join(map(str, wl.dims)), wl.T, wl.true_ranks, wl.noise,
                                  wl.leaf_len, wl.node_ranks, nq, wl.query_kind, wl.theta[0], wl.theta[1],
                                  wl.max_iter, wl.tol),
                   "queries_per_step": nq,
                   "path": "prepared batch: one HIP graph per step, fused Recall+trims+Stitch kernel per LDS bin",
                   "tuning": tuning},
        "sync_batch_ms_per_step": sync_ms,
        "latency_ms": {"batch_p50": ms_per_step, "batch_p99": ms_per_step,
                       "plain_p50": plain["p50_ms"] if plain else None,
                       "plain_p99": plain["p99_ms"] if plain else None},
        "plain_gpu_path": plain,
        "speedup_vs_plain": (qps / plain["queries_per_s"]) if plain else None,
        "appends_per_s": wl.T / build_s,
        "sweeps_mean": float(np.mean(sweeps)),
        "device_us_per_query": {"mean": float(tot.mean()), "p50": float(np.median(tot)), "max": float(tot.max()),
                                "phase_mean": phase_mean, "eig_counters_mean": counters,
                                "timeline": timeline, "slowest": slowest},
        "hits_mean": float(np.mean(hit_counts)),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_detail": traffic_detail,
                     "kernel": "stitch_kernel", "kernel_ms": float(np.mean(kms)),
                     "gflop_per_launch": flops / 1e9},
        "accuracy_vs_oracle": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
