"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP32 arithmetic): hit sets and node ids bit-exact; relative
reconstruction-error difference |e_gpu / e_oracle - 1| <= 1e-5, with e the
error against the raw data in FP64; leading-subspace sine <= 1e-4 on
converged runs; factor orthonormality <= 1e-6.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import recon_bound, compare, level_index, load_store, oracle_tree, recon_diff, round_nodes, say, to_np, ytilde

pytestmark = pytest.mark.gpu

DELTA = 1e-5
SINE = 1e-4
ORTH = 1e-6
# distance of converged reconstructions, |Y^_gpu - Y^_oracle| / |Y^_oracle|: the
# FP32 bar of the error ratio applied to the reconstruction itself, plus the
# Davis-Kahan estimate of what FP32 rounding may move at each mode's rank cut
RECON = 1e-5


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


def test_kernel_parity_tiny_fixed_sweeps(tiny):
    """The oracle's node store (FP32-rounded) loaded into the device store:
    isolates trims + Stitch from the leaf/merge path."""
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    ts, te = synth.queries(wl)
    bad = []
    for sweeps in (1, 3):
        gpu.set_query_iters(sweeps, 0.0)
        worst = [0.0, 0.0, 0.0]
        for a, b in zip(ts.tolist(), te.tolist()):
            assert [(h["node_id"], h["lo"], h["hi"]) for h in gpu.hitset(a, b)] == \
                [(v.id, lo, hi) for v, lo, hi in orc.recall(a, b)]
            r = gpu.query(a, b)
            Go, Uo, info = orc.query(a, b, max_iter=sweeps, tol=0.0)
            G, U = to_np(r)
            d, orth, _, eg, eo = compare(X, a, b, G, U, Go, Uo)
            derr = 0.0
            if info["err_model"] is not None:
                # model error from |Y~|^2 - |G|^2: FP32-stored factors bound
                # the squared relative error to about 1e-6
                derr = abs(r.err_model ** 2 - info["err_model"] ** 2)
            ok = (r.sweeps == info["sweeps"] and d <= DELTA and orth <= ORTH and derr <= 1e-6)
            say("tiny sweeps=%d [%d,%d) hits=%d delta=%.2e orth=%.2e derr2=%.2e e=%.4e %s" %
                (sweeps, a, b, r.n_hits, d, orth, derr, eg, "" if ok else "FAIL"))
            if not ok:
                bad.append((sweeps, a, b, d, orth, derr))
            worst = [max(worst[0], d), max(worst[1], orth), max(worst[2], derr)]
        say("tiny fixed sweeps", sweeps, "worst delta %.2e orth %.2e derr2 %.2e" % tuple(worst))
    assert not bad, bad


def test_kernel_parity_tiny_converged_subspaces(tiny):
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    gpu.set_query_iters(60, 0.0)
    ts, te = synth.queries(wl)
    worst = 0.0
    for a, b in zip(ts.tolist()[:16], te.tolist()[:16]):
        say("tiny converged", a, b)
        r = gpu.query(a, b)
        Go, Uo, _ = orc.query(a, b, max_iter=60, tol=0.0)
        G, U = to_np(r)
        d, orth, sine, _, _ = compare(X, a, b, G, U, Go, Uo, wl.true_ranks, SINE, Yt=ytilde(orc, a, b))
        assert d <= DELTA and orth <= ORTH and sine <= SINE, (a, b, d, orth, sine)
        worst = max(worst, sine)
    say("tiny converged worst sine %.2e" % worst)


def test_single_node_range_is_the_stored_node(tiny):
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    for v in orc.complete_nodes()[::5]:
        k, j = level_index(v)
        r = gpu.query(orc.sigma(v), orc.tau(v))
        core, facs = gpu.read_node(k, j)
        assert r.sweeps == 0
        assert np.array_equal(r.core.cpu().numpy(), core)
        for a, b in zip(r.factors, facs):
            assert np.array_equal(a.cpu().numpy(), b)
        assert np.array_equal(core.astype(np.float64), v.H)


def test_end_to_end_tiny_build(tiny, torch):
    """The device builds its own tree (leaf Tucker-ALS + merges) from raw data."""
    wl, X, _ = tiny
    orc = oracle_tree(wl, X, wl.T)
    gpu = _gpu_tree(wl, wl.T)
    say("tiny build")
    gpu.build(X)
    st = gpu.stats()
    T_b = wl.T // wl.leaf_len
    assert st["blocks"] == T_b and st["merges_total"] == T_b - bin(T_b).count("1")
    assert st["height"] == orc.height() and st["nodes"] == len(orc.nodes)
    worst = 0.0
    from oracle.evaluate import relative_error
    for v in orc.complete_nodes():
        k, j = level_index(v)
        core, facs = gpu.read_node(k, j)
        Xi = X[orc.sigma(v):orc.tau(v)]
        e_g = relative_error(Xi, core.astype(np.float64), [f.astype(np.float64) for f in facs])
        e_o = relative_error(Xi, v.H, v.V)
        d = abs(e_g / e_o - 1.0) if e_o > 0 else e_g
        worst = max(worst, d)
    say("tiny build: worst node delta %.2e" % worst)
    assert worst <= DELTA
    ts, te = synth.queries(wl)
    worst = 0.0
    for a, b in zip(ts.tolist(), te.tolist()):
        r = gpu.query(a, b)
        Go, Uo, _ = orc.query(a, b)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, b, G, U, Go, Uo)
        assert orth <= ORTH
        worst = max(worst, d)
    say("tiny build: worst query delta %.2e" % worst)
    assert worst <= DELTA


def test_append_equals_build(torch):
    wl = synth.get("tiny")
    T = 96
    X = synth.series(wl, 0, T)
    a = _gpu_tree(wl, T)
    b = _gpu_tree(wl, T)
    say("append vs build")
    a.build(X)
    for t in range(T):
        b.append(X[t])
    assert a.stats()["merges_total"] == b.stats()["merges_total"]
    for k in range(0, 5):
        for j in range((T // wl.leaf_len) >> k):
            ca, fa = a.read_node(k, j)
            cb, fb = b.read_node(k, j)
            assert np.array_equal(ca, cb)
            assert all(np.array_equal(x, y) for x, y in zip(fa, fb))


def test_batch_equals_alone(tiny):
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    ts, te = synth.queries(wl)
    say("batch vs alone")
    batch = gpu.query_batch(ts, te)
    for i in range(0, len(ts), 3):
        alone = gpu.query(int(ts[i]), int(te[i]))
        assert np.array_equal(alone.core.cpu().numpy(), batch[i].core.cpu().numpy())
        for x, y in zip(alone.factors, batch[i].factors):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        assert alone.sweeps == batch[i].sweeps


def test_range_errors(tiny):
    from paper_2501_06647_amd import TuckerError
    from paper_2501_06647_amd.tucket import TK_ERANGE
    wl, X, orc = tiny
    gpu = _gpu_tree(wl, wl.T)
    load_store(gpu, orc)
    for a, b in [(0, 0), (3, 2), (-1, 4), (0, wl.T + 1)]:
        with pytest.raises(TuckerError) as e:
            gpu.query(a, b)
        assert e.value.status == TK_ERANGE


def test_plain_workload_full_size_sampled(torch):
    """64x64 x T=4096, leaf 8, ranks 10: both sides build their own trees;
    sampled queries compared (the launch shape of the plain path)."""
    wl = synth.get("plain")
    X = synth.series(wl)
    say("plain: gpu build")
    gpu = _gpu_tree(wl, wl.T)
    gpu.build(X)
    say("plain: oracle build")
    orc = oracle_tree(wl, X, wl.T)
    ts, te = synth.queries(wl, n=24)
    worst = 0.0
    refused = accepted = 0
    for a, b in zip(ts.tolist(), te.tolist()):
        say("plain query", a, b)
        assert [(h["node_id"], h["lo"], h["hi"]) for h in gpu.hitset(a, b)] == \
            [(v.id, lo, hi) for v, lo, hi in orc.recall(a, b)]
        r = gpu.query(a, b)
        pr = gpu.last_profile(0)
        refused += pr["eig_warm_refused"]
        accepted += pr["eig_warm"]
        Go, Uo, _ = orc.query(a, b)
        G, U = to_np(r)
        d, orth, _, eg, eo = compare(X, a, b, G, U, Go, Uo)
        assert orth <= ORTH
        worst = max(worst, d)
    say("plain: worst query delta %.2e; warm-started eigensolves %d accepted, %d refused"
        % (worst, accepted, refused))
    assert worst <= DELTA
    # node ranks (10) above the data's rank (8): no gap after the 10th
    # eigenvalue, so the certificate must refuse the subspace iterations
    # (the full solver then gives the results compared above)
    assert refused > 0
    # converged runs (200 sweeps, tolerance 1e-12 on both sides): leading
    # subspaces and the distance between the two reconstructions
    gpu.set_query_iters(200, 1e-12)
    cts, cte = synth.queries(wl, n=64, seed_offset=9)
    pick = [i for i in range(64) if cte[i] - cts[i] <= 1024][:6]
    worst_sine, worst_y = 0.0, 0.0
    for i in pick:
        a, b = int(cts[i]), int(cte[i])
        r = gpu.query(a, b)
        Go, Uo, info = orc.query(a, b, max_iter=200, tol=1e-12)
        G, U = to_np(r)
        Yt = ytilde(orc, a, b)
        d, orth, sine, _, _ = compare(X, a, b, G, U, Go, Uo, wl.true_ranks, SINE, Yt=Yt)
        dy = recon_diff(G, U, Go, Uo)
        bound = RECON + recon_bound(Yt, Go, Uo)
        say("plain converged [%d,%d) sweeps %d/%d delta=%.2e sine=%.2e recon=%.2e (bar %.2e)"
            % (a, b, r.sweeps, info["sweeps"], d, sine, dy, bound))
        assert d <= DELTA and orth <= ORTH and sine <= SINE and dy <= bound, (a, b, d, orth, sine, dy, bound)
        worst_sine, worst_y = max(worst_sine, sine), max(worst_y, dy)
    say("plain converged: worst sine %.2e, worst reconstruction distance %.2e" % (worst_sine, worst_y))


def test_tail_queries(torch):
    """Ranges ending in the incomplete block: tiny data, 63 complete blocks
    and 3 more slices appended on the device; ranges ending in those slices
    (some inside them) against the oracle's provisional piece, every other
    range unchanged; prepared batches refuse the tail; once the block
    completes the same slot holds the real leaf."""
    from paper_2501_06647_amd import TuckerError
    from paper_2501_06647_amd.tucket import TK_ERANGE
    wl = synth.get("tiny")
    X = synth.series(wl)
    Tc = 63 * wl.leaf_len
    gpu = _gpu_tree(wl, wl.T)
    gpu.build(X[:Tc + 3])
    orc = oracle_tree(wl, X, Tc)
    tail = X[Tc:Tc + 3]
    worst = 0.0
    ranges = [(0, Tc + 3), (100, Tc + 1), (Tc - 2, Tc + 2), (Tc, Tc + 3), (Tc + 1, Tc + 3), (Tc + 2, Tc + 3), (5, 200)]
    res = gpu.query_batch([a for a, _ in ranges], [c for _, c in ranges])
    for (a, c), r in zip(ranges, res):
        Go, Uo, info = orc.query(a, c, tail=tail)
        G, U = to_np(r)
        assert G.shape == Go.shape, (a, c)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH, (a, c, orth)
        worst = max(worst, d)
    say("tail queries: worst delta %.2e over %d ranges" % (worst, len(ranges)))
    assert worst <= DELTA
    with pytest.raises(TuckerError) as e:
        gpu.prepare_batch([0], [Tc + 2])
    assert e.value.status == TK_ERANGE
    # the block completes: slot 63 is the real leaf, stitched as any other
    gpu.append(X[Tc + 3])
    full = oracle_tree(wl, X, Tc + 4)
    for a, c in [(0, Tc + 4), (Tc, Tc + 4), (Tc + 1, Tc + 3)]:
        r = gpu.query(a, c)
        Go, Uo, _ = full.query(a, c)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert d <= DELTA and orth <= ORTH, (a, c, d)
