"""Other numbers of modes than the workloads have: p = 2 (a matrix series)
and p = 5, 6 and 7 (the kernels take two to seven modes), built on the
device and queried, against the oracle.

Bars: every node's relative error within 1e-5 of the oracle's (ratio
form); queries within 1e-5, the same sweep counts, factor orthonormality
<= 1e-6; Tucker-ALS from scratch on raw ranges the same.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import compare, node_delta, oracle_tree, say, to_np
from oracle.evaluate import relative_error
from oracle.tucker import effective_ranks, hooi

pytestmark = pytest.mark.gpu

DELTA = 1e-5
ORTH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("dims,ranks,seed", [
    ((30,), (5, 5), 2000),
    ((6, 5, 4, 3), (3, 3, 2, 2, 2), 2001),
    ((4, 3, 3, 3, 2), (3, 2, 2, 2, 2, 2), 2002),
    ((3, 3, 2, 2, 2, 2), (3, 2, 2, 2, 2, 2, 2), 2003),
])
def test_many_modes_parity(torch, dims, ranks, seed):
    from paper_2501_06647_amd import Tree
    # a two-mode leaf is a leaf_len x D_2 matrix: at leaf length 2 and rank 2
    # every node would be exact, so the matrix series takes leaves of 8
    ell, T_ = (8, 128) if len(dims) == 1 else (2, 64)
    wl = synth.Workload("modes%d" % (len(dims) + 1), dims, T_, ranks, 0.05, ell, ranks, 24, "pairs", seed=seed)
    X = synth.series(wl)
    T = wl.T
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=T)
    gpu.build(X.astype(np.float32))
    orc = oracle_tree(wl, X.astype(np.float32).astype(np.float64), T)
    worst = 0.0
    for v in orc.complete_nodes():
        k = (v.hi - v.lo).bit_length() - 1
        core, facs = gpu.read_node(k, v.lo >> k)
        Xi = X[orc.sigma(v):orc.tau(v)]
        e_g = relative_error(Xi, core.astype(np.float64), [f.astype(np.float64) for f in facs])
        e_o = relative_error(Xi, v.H, v.V)
        worst = max(worst, node_delta(e_g, e_o))
    say("p=%d: worst node delta %.2e over %d nodes" % (len(dims) + 1, worst, len(orc.complete_nodes())))
    assert worst <= DELTA
    ts, te = synth.queries(wl)
    res = gpu.query_batch(ts, te)
    worst = 0.0
    for r, a, c in zip(res, ts.tolist(), te.tolist()):
        Go, Uo, info = orc.query(a, c)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and r.sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    say("p=%d: worst query delta %.2e over %d queries" % (len(dims) + 1, worst, len(ts)))
    assert worst <= DELTA
    raw = gpu.raw_tucker(X.astype(np.float32), ts[:8], te[:8])
    worst = 0.0
    for r, a, c in zip(raw, ts[:8].tolist(), te[:8].tolist()):
        rq = effective_ranks(c - a, wl.dims, wl.node_ranks)
        Go, Uo, info = hooi(X[a:c].astype(np.float32).astype(np.float64), rq, wl.max_iter, wl.tol)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and r.sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    say("p=%d: raw Tucker-ALS worst delta %.2e" % (len(dims) + 1, worst))
    assert worst <= DELTA
    worst = 0.0
    Xd = torch.from_numpy(X.astype(np.float32)).to("cuda:0")
    for a, c in [(0, T), (3, 50), (10, 11)]:
        r = gpu.raw_tucker_stream(Xd, a, c)
        rq = effective_ranks(c - a, wl.dims, wl.node_ranks)
        Go, Uo, info = hooi(X[a:c].astype(np.float32).astype(np.float64), rq, wl.max_iter, wl.tol)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and r.sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    say("p=%d: streaming Tucker-ALS worst delta %.2e" % (len(dims) + 1, worst))
    assert worst <= DELTA


def test_three_modes_large_slices(torch):
    """The many-mode experiment's three-way shape: 1000 x 1000 slices, rank 5,
    leaf 1, over 32 slices.  Every leaf is the truncated SVD of its slice
    (from subspace iteration on the device); the oracle builds its own tree
    (Tucker-ALS leaves through LAPACK's SVD, literal stitches) in worker
    processes.  Bars: every node's relative error within 1e-5 of the
    oracle's, the leaves' non-temporal subspaces within a sine of 1e-4 on
    the rank-5 signal (the gap to the noise is two orders), queries within
    1e-5 with the same sweep counts."""
    import time
    from paper_2501_06647_amd import Tree
    from oracle import pool
    from oracle.evaluate import subspace_sine
    from synth.workloads import d5
    wl = d5(3, T=32)
    T = wl.T
    X = synth.series(wl)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=T)
    Xd = torch.from_numpy(X.astype(np.float32)).to("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpu.build(Xd)
    torch.cuda.synchronize()
    say("p=3 1000x1000: built %d slices in %.3f s" % (T, time.perf_counter() - t0))
    orc = pool.lazy_tree(wl, T)
    pool.fill(orc, wl, 2, range(T // 4))
    worst, worst_sine, n = 0.0, 0.0, 0
    for k in range(6):
        for j in range(T >> k):
            v = orc.node(k, j)
            orc.ensure(v)
            core, facs = gpu.read_node(k, j)
            Xi = X[orc.sigma(v):orc.tau(v)]
            e_g = relative_error(Xi, core.astype(np.float64), [f.astype(np.float64) for f in facs])
            e_o = relative_error(Xi, v.H, v.V)
            worst = max(worst, abs(e_g / e_o - 1.0))
            if k == 0:
                for m in (1, 2):
                    worst_sine = max(worst_sine, subspace_sine(v.V[m], facs[m].astype(np.float64), 5))
            n += 1
    say("p=3 1000x1000: worst node delta %.2e over %d nodes, worst leaf sine %.2e" % (worst, n, worst_sine))
    assert worst <= DELTA and worst_sine <= 1e-4
    ts, te = synth.queries(wl)
    ts, te = ts[:16], te[:16]
    res = gpu.query_batch(ts, te)
    worst = 0.0
    for r, a, c in zip(res, ts.tolist(), te.tolist()):
        Go, Uo, info = orc.query(a, c)
        G, U = to_np(r)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert orth <= ORTH and r.sweeps == info["sweeps"], (a, c)
        worst = max(worst, d)
    say("p=3 1000x1000: worst query delta %.2e over %d queries" % (worst, len(ts)))
    assert worst <= DELTA
