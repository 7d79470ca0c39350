"""Prepared batches (graph replay, device Recall), launch tunings, the
autotuner and the serving engine, through the C ABI.

Bars: hit sets bit-exact against the oracle's Recall; every prepared-batch
replay bit-identical to the synchronous batch; every tuning within the FP32
parity tolerance of the oracle; a served query bit-identical to the same
query run alone on a tree holding the same slices.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import compare, level_index, load_store, oracle_tree, round_nodes, say, to_np
from oracle import stitch as ostitch
from oracle.tree import StreamSegmentTree
from oracle.tucker import effective_ranks

pytestmark = pytest.mark.gpu

DELTA = 1e-5
ORTH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu_tree(wl, T, **kw):
    from paper_2501_06647_amd import Tree
    args = dict(max_iter=wl.max_iter, tol=wl.tol)
    args.update(kw)
    return Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, capacity_T=T, **args)


@pytest.fixture(scope="module")
def tiny(torch):
    wl = synth.get("tiny")
    X = synth.series(wl)
    orc = oracle_tree(wl, X, wl.T)
    round_nodes(orc)
    return wl, X, orc


def _same(a, b):
    """Bitwise equality of two query results."""
    if not np.array_equal(a.core.cpu().numpy(), b.core.cpu().numpy()):
        return False
    return all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a.factors, b.factors)) \
        and a.sweeps == b.sweeps


def _structure_oracle(wl, T):
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol)
    for _ in range(T // wl.leaf_len):
        t.append(None)
    return t


def test_device_recall_matches_oracle(tiny, torch):
    """The fused kernel's own Recall (written back per query) equals the
    oracle's hit set, on the tiny tree and on the plain tree's 2048 queries."""
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    ts, te = synth.queries(wl)
    b = gpu.prepare_batch(ts, te)
    b.run()
    for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
        got = [(h["node_id"], h["lo"], h["hi"], h["partial"]) for h in b.device_hits(i)]
        want = [(v.id, lo, hi, (lo, hi) != (orc.sigma(v), orc.tau(v))) for v, lo, hi in orc.recall(a, c)]
        assert got == want, (a, c, got, want)
    b.close()
    # plain shape: structure-only oracle, GPU tree restored to the full horizon
    wp = synth.get("plain")
    so = _structure_oracle(wp, wp.T)
    g2 = _gpu_tree(wp, wp.T)
    g2.build(synth.series(wp))
    ts, te = synth.queries(wp)
    g2.set_query_iters(1, 0.0)
    b2 = g2.prepare_batch(ts, te)
    b2.run()
    bad = 0
    for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
        got = [(h["node_id"], h["lo"], h["hi"]) for h in b2.device_hits(i)]
        want = [(v.id, lo, hi) for v, lo, hi in so.recall(a, c)]
        bad += got != want
    say("plain device recall: %d mismatches of %d" % (bad, len(ts)))
    assert bad == 0


def test_graph_replays_equal_sync_batch(tiny, torch):
    """Each replay of the captured graph, with unrelated eager device work
    and host synchronisations between replays, reproduces the synchronous
    batch bit for bit."""
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    ts, te = synth.queries(wl)
    ref = gpu.query_batch(ts, te)
    b = gpu.prepare_batch(ts, te)
    for rep in range(4):
        for x in b.outputs:
            x[0].fill_(0.0)
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
        b.run()
        got = b.results()
        bad = [i for i in range(len(ts)) if not _same(got[i], ref[i])]
        say("replay %d: %d mismatches, kernel %.3f ms" % (rep, len(bad), b.kernel_ms()))
        assert not bad, bad
    b.close()


@pytest.mark.parametrize("tuning", [
    dict(wide_threshold=16, wide_threads=128, persistent=1),
    dict(wide_threshold=16, wide_threads=256, persistent=0),
    dict(wide_threshold=32, wide_threads=256, persistent=1, graph=0),
    dict(wide_threshold=96, wide_threads=128, persistent=1),
    dict(basis_pct=1),    # every mode in its full coordinates
    dict(basis_pct=100),  # the span basis whenever it is smaller
    dict(wide_threshold=16, lds_n=16, rest_threads=256),  # most jobs above the LDS cap, 256 threads
    dict(wide_core=64),  # every tiny core (125 elements) in wide workgroups
])
def test_tunings_keep_parity(tiny, tuning):
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    gpu.set_tuning(**tuning)
    gpu.set_query_iters(3, 0.0)
    ts, te = synth.queries(wl)
    b = gpu.prepare_batch(ts, te)
    b.run()
    res = b.results()
    worst = 0.0
    for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
        Go, Uo, info = orc.query(a, c, max_iter=3, tol=0.0)
        G, U = to_np(res[i])
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert res[i].sweeps == info["sweeps"] and orth <= ORTH, (a, c, orth)
        worst = max(worst, d)
    say("tuning %s: worst delta %.2e" % (tuning, worst))
    assert worst <= DELTA
    b.close()


def test_query_output_ranks(tiny, torch):
    """Queries at output ranks (3, 3, 3) below the nodes' (5, 5, 5): the
    tiny workload's query list plus two stored nodes' own ranges (which the
    stitch then runs on one entire hit), against the oracle's query at the
    same ranks, three sweeps each; back at the nodes' ranks such a range is
    the stored node again (no sweeps)."""
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    gpu.set_query_ranks((3, 3, 3))
    gpu.set_query_iters(3, 0.0)
    ts, te = synth.queries(wl)
    ts = np.concatenate([ts, [0, 128]])
    te = np.concatenate([te, [64, 192]])
    b = gpu.prepare_batch(ts, te)
    b.run()
    res = b.results()
    worst = 0.0
    for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
        Go, Uo, info = orc.query(a, c, max_iter=3, tol=0.0, ranks=(3, 3, 3))
        G, U = to_np(res[i])
        assert G.shape == Go.shape, (a, c, G.shape, Go.shape)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert res[i].sweeps == info["sweeps"] and orth <= ORTH, (a, c, orth)
        worst = max(worst, d)
    say("output ranks (3, 3, 3): worst delta %.2e over %d queries" % (worst, len(ts)))
    assert worst <= DELTA
    b.close()
    gpu.set_query_ranks(None)
    r = gpu.query(0, 64)
    assert r.sweeps == 0 and tuple(r.ranks) == (5, 5, 5)


@pytest.mark.parametrize("theta", [(1, 2), (9, 10), (1, 1)])
def test_theta_sweep_parity(tiny, torch, theta):
    """Alg. "recall" at other thresholds (the theta sweep of the paper's
    efficiency-accuracy comparison).  Nodes do not depend on theta, so the
    tiny store is loaded into a tree of that theta: device hit sets
    bit-exact against the oracle's Recall at the same theta, results within
    the FP32 tolerance (three sweeps)."""
    from paper_2501_06647_amd import Tree
    wl, X, orc = tiny
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    load_store(gpu, orc)
    gpu.set_query_iters(3, 0.0)
    saved = orc.theta
    orc.theta = theta
    try:
        ts, te = synth.queries(wl)
        b = gpu.prepare_batch(ts, te)
        b.run()
        res = b.results()
        worst, hits = 0.0, 0
        for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
            want = orc.recall(a, c)
            got = [(h["node_id"], h["lo"], h["hi"]) for h in b.device_hits(i)]
            assert got == [(v.id, lo, hi) for v, lo, hi in want], (a, c)
            hits += len(want)
            Go, Uo, info = orc.query(a, c, max_iter=3, tol=0.0)
            G, U = to_np(res[i])
            d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
            assert orth <= ORTH and res[i].sweeps == info["sweeps"], (a, c)
            worst = max(worst, d)
        say("theta %d/%d: %.2f hits per query, worst delta %.2e" % (theta[0], theta[1], hits / len(ts), worst))
        assert worst <= DELTA
        b.close()
    finally:
        orc.theta = saved


def test_fixed_block_parity(tiny, torch):
    """The fixed-block hit set (level 2: blocks of 16 slices), queries on
    host-planned hits: on the full tiny store, hit sets (host and device)
    bit-exact against the oracle's and results within the FP32 tolerance;
    on the store cut to 200 slices (12 complete blocks, the rest from Alg.
    "recall"), the same against a 50-block oracle tree holding the same
    nodes."""
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    gpu.set_query_iters(3, 0.0)
    gpu.set_query_recall(2)
    ts, te = synth.queries(wl)
    b = gpu.prepare_batch(ts, te)
    b.run()
    res = b.results()
    worst = 0.0
    for i, (a, c) in enumerate(zip(ts.tolist(), te.tolist())):
        want = [(v.id, lo, hi) for v, lo, hi in orc.fixed_block_hits(a, c, 2)]
        assert [(h["node_id"], h["lo"], h["hi"]) for h in b.device_hits(i)] == want, (a, c)
        assert [(h["node_id"], h["lo"], h["hi"]) for h in gpu.hitset(a, c)] == want, (a, c)
        Go, Uo, info = orc.query(a, c, max_iter=3, tol=0.0, level=2)
        G, U = to_np(res[i])
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and res[i].sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    b.close()
    # the store cut to 50 blocks: the last 8 slices come from Alg. "recall"
    T50 = 200
    g50 = _gpu_tree(wl, wl.T)
    g50.restore_begin(T50)
    by_range = {}
    for v in orc.complete_nodes():
        if v.hi <= T50 // wl.leaf_len:
            k, j = level_index(v)
            g50.load_node(k, j, v.H, v.V)
            by_range[(v.lo, v.hi)] = v
    g50.set_query_iters(3, 0.0)
    g50.set_query_recall(2)
    so = _structure_oracle(wl, T50)
    rng = np.random.default_rng(11)
    pairs = [(int(a), T50) for a in rng.choice(T50, size=6, replace=False)] + [(190, 199), (3, 196)]
    for a, c in pairs:
        hits = so.fixed_block_hits(a, c, 2)
        got = [(h["node_id"], h["lo"], h["hi"]) for h in g50.hitset(a, c)]
        assert got == [(v.id, lo, hi) for v, lo, hi in hits], (a, c)
        pieces = []
        for v, lo, hi in hits:
            node = by_range[(v.lo, v.hi)]
            if lo == so.sigma(v) and hi == so.tau(v):
                pieces.append(ostitch.Piece(node.H, list(node.V)))
            else:
                pieces.append(ostitch.trim(node.H, node.V, lo - so.sigma(v), hi - lo))
        r = g50.query(a, c)
        if len(hits) == 1 and hits[0][1] == so.sigma(hits[0][0]) and hits[0][2] == so.tau(hits[0][0]):
            continue
        Go, Uo, info = ostitch.stitch(pieces, effective_ranks(c - a, wl.dims, wl.node_ranks), 3, 0.0)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and r.sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    say("fixed blocks (level 2): worst delta %.2e" % worst)
    assert worst <= DELTA


def test_autotune_picks_a_valid_tuning(torch):
    wl = synth.get("plain")
    T = 1024
    X = synth.series(wl, 0, T)
    gpu = _gpu_tree(wl, T)
    gpu.build(X)
    ts, te = synth.queries(wl, T=T, n=128)
    best, ms = gpu.autotune(ts, te, reps=1)
    say("autotune:", best, "%.3f ms" % ms)
    assert best == gpu.tuning() and ms > 0
    assert best["wide_threshold"] in (32, 48, 64, 96) and best["wide_threads"] in (128, 256)


def _serve_and_check(wl, X, T0, T1, n_every, burst, torch, max_batch=0, seed=7):
    """Serve appends X[T0:T1] with a query every n_every appends (random
    ranges inside the submitter's snapshot) plus a burst of queries; compare
    every result bitwise with the same query on a reference tree restored to
    that snapshot, and every node of the served tree with the reference."""
    rng = np.random.default_rng(seed)
    ref = _gpu_tree(wl, T1)
    ref.build(X[:T1])
    srv_tree = _gpu_tree(wl, T1)
    srv_tree.build(X[:T0])
    srv = srv_tree.serve(max_batch=max_batch)
    ell = wl.leaf_len
    issued = []

    def submit_query(T):
        Tc = (T // ell) * ell
        a, c = sorted(rng.choice(Tc + 1, size=2, replace=False).tolist())
        issued.append((srv.submit_query(a, c), a, c, Tc))

    T = T0
    for t in range(T0, T1):
        srv.submit_append(X[t])
        T += 1
        if (t - T0) % n_every == 0:
            submit_query(T)
        if t == (T0 + T1) // 2:
            for _ in range(burst):
                submit_query(T)
    srv.sync()
    stats = srv.stats()
    say("serve stats:", stats)
    results = [(srv.result(tk), a, c, Tc) for tk, a, c, Tc in issued]
    lat = [srv.times(tk) for tk, _, _, _ in issued]
    srv.stop()
    assert stats["completed"] == stats["queries"] + stats["appends"]
    assert stats["max_batch_seen"] > 1, "no batch admitted more than one query"
    bad = 0
    for Tc in sorted(set(r[3] for r in results)):
        ref.restore_begin(Tc)
        for r, a, c, Tq in results:
            if Tq != Tc:
                continue
            alone = ref.query(a, c)
            if not _same(r, alone):
                bad += 1
                say("mismatch [%d,%d) at T_c=%d" % (a, c, Tc))
    ref.restore_begin(T1)
    nodes_bad = 0
    st = srv_tree.stats()
    assert st["T"] == T1 and st["blocks"] == T1 // ell
    for k in range(0, 20):
        n = (T1 // ell) >> k
        if n == 0:
            break
        for j in range(n):
            ca, fa = srv_tree.read_node(k, j)
            cb, fb = ref.read_node(k, j)
            if not (np.array_equal(ca, cb) and all(np.array_equal(x, y) for x, y in zip(fa, fb))):
                nodes_bad += 1
    wait = np.array([l[2] - l[0] for l in lat])
    say("served %d queries: %d mismatches, %d node mismatches; latency p50 %.0f us p99 %.0f us"
        % (len(results), bad, nodes_bad, np.percentile(wait, 50), np.percentile(wait, 99)))
    assert bad == 0 and nodes_bad == 0


def test_serving_tiny_alone_equals_mix(torch):
    wl = synth.get("tiny")
    X = synth.series(wl)
    _serve_and_check(wl, X, 64, wl.T, 3, 48, torch, max_batch=16)


def test_serving_plain_alone_equals_mix(torch):
    wl = synth.get("plain")
    X = synth.series(wl, 0, 2560)
    _serve_and_check(wl, X, 2048, 2560, 4, 96, torch)


def test_serving_admission_and_exclusion(torch):
    from paper_2501_06647_amd import TuckerError
    from paper_2501_06647_amd.tucket import TK_EBUSY, TK_ENOMEM, TK_ERANGE
    wl = synth.get("plain")
    T = 1024
    gpu = _gpu_tree(wl, T)
    gpu.build(synth.series(wl, 0, T))
    ts, te = synth.queries(wl, T=T, n=64)
    ws = [gpu.query_shape(int(a), int(b)).ws_bytes for a, b in zip(ts, te)]
    i_small, i_big = int(np.argmin(ws)), int(np.argmax(ws))
    small, big = ws[i_small], ws[i_big]
    # a budget that admits the small query; the big one exceeds it even with
    # its eigen buffer (< 70 KB at these ranks) in LDS
    assert big - 70000 > small, (small, big)
    srv = gpu.serve(ws_budget_bytes=3 * small)
    try:
        with pytest.raises(TuckerError) as e:
            gpu.query(0, 8)
        assert e.value.status == TK_EBUSY
        with pytest.raises(TuckerError) as e:
            srv.submit_query(0, T + 1)
        assert e.value.status == TK_ERANGE
        with pytest.raises(TuckerError) as e:
            srv.submit_query(int(ts[i_big]), int(te[i_big]))
        assert e.value.status == TK_ENOMEM
        t = srv.submit_query(int(ts[i_small]), int(te[i_small]))
        srv.wait(t)
        assert srv.poll(t)
        assert srv.stats()["rejected"] == 1
    finally:
        srv.stop()
    r = gpu.query(0, 8)  # synchronous calls work again
    assert r.n_hits >= 1


def _oracle_at(wl, Tc, memo):
    """An on-demand oracle tree at committed horizon Tc whose nodes come from
    memo ((level, index) -> (H, V), all built by the oracle from raw data)."""
    from oracle import pool
    from oracle.tree import node_key
    t = pool.lazy_tree(wl, Tc)
    for v in t.complete_nodes():
        H, V = memo[node_key(v)]
        v.H, v.V = H, list(V)
    return t


def test_serving_shape_results_against_oracle(torch):
    """The serving workload's shape (128 x 128 slices, drifting rank-16
    model, leaf 1, node ranks 16): a tree of 1024 slices serves 512 more
    appended one at a time, interleaved with queries of log-uniform lengths
    inside each query's snapshot, first with FP32 queries, then (a second
    session) with BF16 queries; merges are FP32 throughout.  Sampled served
    results are compared with the oracle at their snapshots, the oracle
    building every node itself from the raw slices."""
    import math
    from oracle import pool
    from oracle.tree import node_key
    from paper_2501_06647_amd.tucket import TK_BF16
    wl = synth.get("serving")
    T0, T1, T2 = 1024, 1280, 1536
    X = synth.series(wl, 0, T2)
    gpu = _gpu_tree(wl, T2)
    gpu.build(X[:T0])
    rng = np.random.default_rng(23)
    served = []
    for prec, t_lo, t_hi in ((None, T0, T1), (TK_BF16, T1, T2)):
        if prec is not None:
            gpu.set_query_prec(prec)
        srv = gpu.serve(max_batch=64)
        T = t_lo
        tickets = []
        for t in range(t_lo, t_hi):
            srv.submit_append(X[t])
            T += 1
            if t % 4 == 0:
                L = int(min(T, max(1, math.floor(math.exp(rng.uniform(0.0, math.log(T)))))))
                a = int(rng.integers(0, T - L + 1))
                tickets.append((srv.submit_query(a, a + L), a, a + L, T))
        srv.sync()
        st = srv.stats()
        say("serving session prec=%s: %s" % (prec, st))
        assert st["completed"] == st["queries"] + st["appends"]
        pick = rng.choice(len(tickets), size=min(10, len(tickets)), replace=False)
        for i in sorted(pick.tolist()):
            tk, a, c, Tc = tickets[i]
            r = srv.result(tk)
            served.append((prec, a, c, Tc, to_np(r)))
        srv.stop()
    # the oracle's own nodes over [0, T2)
    orc = pool.lazy_tree(wl, T2)
    level = pool.pool_level(wl)
    pool.fill(orc, wl, level, range(T2 // (wl.leaf_len << level)))
    for v in orc.complete_nodes():
        orc.ensure(v)
    memo = {node_key(v): (v.H, v.V) for v in orc.complete_nodes()}
    worst = {None: 0.0, TK_BF16: 0.0}
    for prec, a, c, Tc, (G, U) in served:
        o = _oracle_at(wl, Tc, memo)
        Go, Uo, info = o.query(a, c)
        d, orth, _, eg, _ = compare(X, a, c, G, U, Go, Uo)
        say("served prec=%s [%d,%d) at T_c=%d hits=%d delta=%.2e orth=%.2e e=%.4e"
            % (prec, a, c, Tc, len(info["hits"]), d, orth, eg))
        assert orth <= ORTH
        worst[prec] = max(worst[prec], d)
    say("served vs oracle: worst delta FP32 %.2e (bar 1e-5), BF16 %.2e (bar 1e-2)" % (worst[None], worst[TK_BF16]))
    assert worst[None] <= DELTA and worst[TK_BF16] <= 1e-2
