"""tk_query_noalloc (the entry point that allocates nothing) against
tk_query: the same kernels on the same tree, so the results must be
identical bit for bit; two calls in a row, the second with a smaller
range (the scratch keeps the first call's contents), each in a fresh
output buffer and again into the first call's buffers.  Also checked
against the oracle to the parity bar, and the argument and size checks."""

import numpy as np
import pytest

import synth
from gpu_helpers import compare, oracle_tree, say, to_np

pytestmark = pytest.mark.gpu


def _same(a, b):
    return (np.array_equal(a.core.cpu().numpy(), b.core.cpu().numpy())
            and all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a.factors, b.factors))
            and a.sweeps == b.sweeps and a.ranks == b.ranks)


def test_noalloc_query_equals_query():
    import torch
    from paper_2501_06647_amd import Tree, TuckerError
    from paper_2501_06647_amd.tucket import TK_ERANGE
    assert torch.cuda.is_available()
    wl = synth.get("plain")
    T = 1024
    X = synth.series(wl, 0, T)
    tree = Tree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol, capacity_T=T)
    tree.build(X)
    orc = oracle_tree(wl, X, T)
    first = None
    for a, b in [(3, 1000), (17, 300)]:  # the second range is smaller
        say("noalloc [%d, %d)" % (a, b))
        ref = tree.query(a, b)
        got = tree.query_noalloc(a, b)
        assert _same(ref, got), (a, b)
        if first is not None:  # into the first call's (larger) buffers: shapes differ, so fresh ones
            again = tree.query_noalloc(a, b)
            assert _same(ref, again)
        first = got
        Go, Uo, _ = orc.query(a, b)
        G, U = to_np(got)
        d, orth, _, _, _ = compare(X, a, b, G, U, Go, Uo)
        say("noalloc [%d, %d) delta %.2e orth %.2e" % (a, b, d, orth))
        assert d <= 1e-5 and orth <= 1e-6
    # the same range twice into the same output buffers
    r1 = tree.query_noalloc(40, 900)
    r2 = tree.query_noalloc(40, 900, out=r1)
    assert _same(tree.query(40, 900), r2)
    with pytest.raises(TuckerError) as e:
        tree.query_noalloc(5, T + 1)
    assert e.value.status == TK_ERANGE
    with pytest.raises(TuckerError) as e:
        tree.query_noalloc(9, 9)
    assert e.value.status == TK_ERANGE
