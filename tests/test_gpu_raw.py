"""Tucker-ALS from scratch on raw ranges (tk_raw_tucker, one workgroup per
range, and tk_raw_tucker_stream, many workgroups per range): the accuracy
reference and naive baseline of the paper's comparisons, against the
oracle's Tucker-ALS on the same FP32 data.

Bars: |e_gpu / e_oracle - 1| <= 1e-5, e the relative error against the
raw data; the same sweep counts; factor orthonormality <= 1e-6.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import compare, say, to_np
from oracle.tucker import effective_ranks, hooi

pytestmark = pytest.mark.gpu

DELTA = 1e-5
ORTH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _check(gpu, wl, X, ranges, ranks, max_iter, tol):
    X32 = X.astype(np.float32)
    ts = np.array([a for a, _ in ranges], dtype=np.int64)
    te = np.array([c for _, c in ranges], dtype=np.int64)
    res = gpu.raw_tucker(X32, ts, te)
    worst = 0.0
    for (a, c), r in zip(ranges, res):
        rq = effective_ranks(c - a, wl.dims, ranks)
        Go, Uo, info = hooi(X32[a:c].astype(np.float64), rq, max_iter, tol)
        G, U = to_np(r)
        assert G.shape == tuple(rq), (a, c, G.shape, rq)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert r.sweeps == info["sweeps"] and orth <= ORTH, (a, c, r.sweeps, info["sweeps"], orth)
        worst = max(worst, d)
    return worst


def test_raw_tucker_tiny(torch):
    """Every tiny query range plus single slices and ranges shorter than the
    temporal rank; then at output ranks (3, 3, 3)."""
    from paper_2501_06647_amd import Tree
    wl = synth.get("tiny")
    X = synth.series(wl)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    ts, te = synth.queries(wl)
    ranges = [(int(a), int(c)) for a, c in zip(ts, te)] + [(0, 1), (17, 20), (0, wl.T)]
    worst = _check(gpu, wl, X, ranges, wl.node_ranks, wl.max_iter, wl.tol)
    say("raw Tucker-ALS tiny: worst delta %.2e over %d ranges" % (worst, len(ranges)))
    assert worst <= DELTA
    gpu.set_query_ranks((3, 3, 3))
    worst = _check(gpu, wl, X, ranges[:12], (3, 3, 3), wl.max_iter, wl.tol)
    say("raw Tucker-ALS tiny at ranks (3, 3, 3): worst delta %.2e" % worst)
    assert worst <= DELTA


def test_raw_tucker_plain_shapes(torch):
    """Plain-workload ranges up to the whole series (4096 x 64 x 64), several
    in one launch."""
    from paper_2501_06647_amd import Tree
    wl = synth.get("plain")
    X = synth.series(wl)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    ranges = [(0, wl.T), (1000, 3001), (5, 13), (4090, 4096), (777, 1300)]
    worst = _check(gpu, wl, X, ranges, wl.node_ranks, wl.max_iter, wl.tol)
    say("raw Tucker-ALS plain: worst delta %.2e over %d ranges" % (worst, len(ranges)))
    assert worst <= DELTA


def _check_stream(gpu, wl, X, ranges, ranks, max_iter, tol):
    import torch
    Xd = torch.from_numpy(X.astype(np.float32)).to("cuda:0")
    worst = 0.0
    for a, c in ranges:
        r = gpu.raw_tucker_stream(Xd, a, c)
        rq = effective_ranks(c - a, wl.dims, ranks)
        Go, Uo, info = hooi(X[a:c].astype(np.float32).astype(np.float64), rq, max_iter, tol)
        G, U = to_np(r)
        assert G.shape == tuple(rq), (a, c, G.shape, rq)
        d, orth, _, _, _ = compare(X, a, c, G, U, Go, Uo)
        assert r.sweeps == info["sweeps"] and orth <= ORTH, (a, c, r.sweeps, info["sweeps"], orth)
        worst = max(worst, d)
    return worst


def test_raw_tucker_stream_tiny_and_plain(torch):
    """The many-workgroup Tucker-ALS (tk_raw_tucker_stream): tiny ranges
    down to one slice (one span each, spans of one slice) and at ranks
    (3, 3, 3); plain ranges up to the whole series, with a ragged last span
    (3997 slices: 500 spans of 8, the last of 5)."""
    from paper_2501_06647_amd import Tree
    wl = synth.get("tiny")
    X = synth.series(wl)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    ranges = [(0, 1), (17, 20), (3, 70), (0, wl.T)]
    worst = _check_stream(gpu, wl, X, ranges, wl.node_ranks, wl.max_iter, wl.tol)
    gpu.set_query_ranks((3, 3, 3))
    worst = max(worst, _check_stream(gpu, wl, X, ranges, (3, 3, 3), wl.max_iter, wl.tol))
    say("streaming Tucker-ALS tiny: worst delta %.2e" % worst)
    assert worst <= DELTA
    gpu.close()
    wl = synth.get("plain")
    X = synth.series(wl)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    ranges = [(0, wl.T), (3, 4000), (5, 13), (777, 1300)]
    worst = _check_stream(gpu, wl, X, ranges, wl.node_ranks, wl.max_iter, wl.tol)
    say("streaming Tucker-ALS plain: worst delta %.2e over %d ranges" % (worst, len(ranges)))
    assert worst <= DELTA
    # the same decomposition as the one-workgroup kernel, to rounding
    one = gpu.raw_tucker(X.astype(np.float32), np.array([3]), np.array([4000]))[0]
    many = gpu.raw_tucker_stream(X.astype(np.float32), 3, 4000)
    d, _, _, _, _ = compare(X, 3, 4000, *to_np(many), *to_np(one))
    say("streaming vs one-workgroup Tucker-ALS on [3, 4000): delta %.2e" % d)
    assert d <= DELTA and many.sweeps == one.sweeps


def test_raw_tucker_stream_batch_workload(torch):
    """The batch workload (128 x 96 slices, ranks 16) on 8000 slices (512
    spans of 16, the last ragged) against the oracle's Tucker-ALS."""
    from paper_2501_06647_amd import Tree
    wl = synth.get("batch")
    X = synth.series(wl, 0, 9000)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    worst = _check_stream(gpu, wl, X, [(1000, 9000)], wl.node_ranks, wl.max_iter, wl.tol)
    say("streaming Tucker-ALS batch workload, 8000 slices: delta %.2e" % worst)
    assert worst <= DELTA


def test_raw_tucker_stream_four_modes(torch):
    """The precision workload's four-way shape (200 x 24 x 8 slices, ranks
    (20, 20, 6, 4), R_1 = 480) on 1000 slices against the oracle."""
    from paper_2501_06647_amd import Tree
    wl = synth.get("precision")
    X = synth.series(wl, 0, 1200)
    gpu = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=wl.max_iter, tol=wl.tol, capacity_T=wl.T)
    worst = _check_stream(gpu, wl, X, [(100, 1100), (0, 37)], wl.node_ranks, wl.max_iter, wl.tol)
    say("streaming Tucker-ALS precision workload: delta %.2e" % worst)
    assert worst <= DELTA
