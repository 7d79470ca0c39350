"""The oracle's on-demand tree against its eager tree.

A node's decomposition depends only on the slices under it, so a tree that
decomposes nodes when a query first needs them, or that takes the nodes of a
subtree from an eager tree built over that subtree's slices alone, must hold
exactly (bit for bit) what the eager tree holds.  These checks are what lets
the full-size parity tests run the oracle on sampled queries of long series.
"""

import numpy as np
import pytest

import synth
from oracle.tree import LazyStreamSegmentTree, StreamSegmentTree, node_key


def _eager(wl, X, nblocks, base=0):
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol)
    ell = wl.leaf_len
    for b in range(nblocks):
        t.append(X[(base + b) * ell:(base + b + 1) * ell])
    return t


def _lazy(wl, X, nblocks):
    t = LazyStreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol,
                              source=lambda a, b: X[a:b])
    t.append_blocks(nblocks)
    return t


@pytest.mark.parametrize("nblocks", [37, 64])
def test_lazy_queries_equal_eager(nblocks):
    wl = synth.get("tiny")
    X = synth.series(wl, 0, nblocks * wl.leaf_len)
    eager = _eager(wl, X, nblocks)
    lazy = _lazy(wl, X, nblocks)
    T = nblocks * wl.leaf_len
    ts, te = synth.queries(wl, T=T, n=12)
    for a, c in list(zip(ts.tolist(), te.tolist())) + [(0, T), (3, 4)]:
        Ge, Ue, ie = eager.query(a, c)
        Gl, Ul, il = lazy.query(a, c)
        assert [(v.id, lo, hi) for v, lo, hi in ie["hits"]] == [(v.id, lo, hi) for v, lo, hi in il["hits"]]
        assert np.array_equal(Ge, Gl)
        assert all(np.array_equal(x, y) for x, y in zip(Ue, Ul))
    # only the nodes under some hit were decomposed
    made = [v for v in lazy.complete_nodes() if v.H is not None]
    assert 0 < len(made) <= len(lazy.complete_nodes())


def test_subtree_nodes_equal_standalone_tree():
    """The nodes of the subtree over blocks [16, 32) equal those of an eager
    tree built from those 16 blocks alone (index shifted by 16 >> level)."""
    wl = synth.get("tiny")
    X = synth.series(wl, 0, 48 * wl.leaf_len)
    eager = _eager(wl, X, 48)
    part = _eager(wl, X, 16, base=16)
    full = {node_key(v): v for v in eager.complete_nodes()}
    n = 0
    for v in part.complete_nodes():
        k, j = node_key(v)
        w = full[(k, j + (16 >> k))]
        assert np.array_equal(v.H, w.H) and all(np.array_equal(x, y) for x, y in zip(v.V, w.V))
        n += 1
    assert n == 31


def test_put_then_lazy_rest_equals_eager():
    wl = synth.get("tiny")
    X = synth.series(wl, 0, 32 * wl.leaf_len)
    eager = _eager(wl, X, 32)
    lazy = _lazy(wl, X, 32)
    for base in (0, 8):
        part = _eager(wl, X, 8, base=base)
        for v in part.complete_nodes():
            k, j = node_key(v)
            lazy.put(k, j + (base >> k), v.H, v.V)
    G1, U1, _ = eager.query(0, 128)
    G2, U2, _ = lazy.query(0, 128)
    assert np.array_equal(G1, G2) and all(np.array_equal(x, y) for x, y in zip(U1, U2))


def test_worker_subtrees_equal_eager():
    """The test-side pool (subtrees built in spawned workers) fills the
    on-demand tree with exactly the eager tree's nodes."""
    from oracle import pool as oracle_pool
    wl = synth.get("tiny")
    nb = 64
    X = synth.series(wl, 0, nb * wl.leaf_len)
    eager = _eager(wl, X, nb)
    lazy = oracle_pool.lazy_tree(wl, nb * wl.leaf_len)
    oracle_pool.fill(lazy, wl, 4, [0, 2, 3])
    made = {node_key(v): v for v in lazy.complete_nodes() if v.H is not None}
    assert len(made) == 3 * 31
    full = {node_key(v): v for v in eager.complete_nodes()}
    for key, v in made.items():
        assert np.array_equal(v.H, full[key].H) and all(np.array_equal(x, y) for x, y in zip(v.V, full[key].V))
    G1, U1, _ = eager.query(5, 250)
    G2, U2, _ = lazy.query(5, 250)
    assert np.array_equal(G1, G2) and all(np.array_equal(x, y) for x, y in zip(U1, U2))


def test_any_slice_range_of_large_slices_matches_the_whole(monkeypatch):
    """Large slices draw their noise in chunks of fewer slices; a range cut
    anywhere equals the same rows of the whole series (what the worker
    processes and the on-demand tree rely on)."""
    from synth import workloads
    monkeypatch.setattr(workloads, "NOISE_CHUNK_ELEMS", 3 * 20 * 20)
    wl = synth.Workload("chunks", (20, 20), 40, (3, 3, 3), 0.1, 1, (3, 3, 3), 4, "pairs", seed=77)
    assert workloads._noise_chunk(wl) == 3
    X = synth.series(wl)
    for a, b in ((0, 40), (1, 2), (2, 7), (5, 6), (17, 40)):
        np.testing.assert_array_equal(synth.series(wl, a, b), X[a:b])
