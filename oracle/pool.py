"""Oracle nodes for long series, built in worker processes.

TEST INFRASTRUCTURE ONLY (like the rest of this package): used by the
full-size parity tests and the benchmark's oracle leg.

The oracle decomposes a node from the slices under it only, so the subtrees
of one tree level are independent: each worker builds an eager oracle tree
over one subtree's blocks (``synth`` regenerates any slice range on its
own), and the parent stores the nodes in an on-demand oracle tree, which
makes whatever is still missing (the nodes above the subtrees, short hits)
itself.  Nothing here computes a decomposition: the workers and the parent
run the oracle's own code.  Workers are spawned (no inherited GPU state)
and each uses one BLAS thread.
"""

import multiprocessing as mp
import os


def _subtree(args):
    name, level, index = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        import synth
        from oracle.tree import StreamSegmentTree, node_key
        wl = synth.get(name)
        ell = wl.leaf_len
        nb = 1 << level
        b0 = index * nb
        X = synth.series(wl, b0 * ell, (b0 + nb) * ell)
        t = StreamSegmentTree(wl.dims, wl.node_ranks, ell, wl.theta, wl.max_iter, wl.tol)
        for b in range(nb):
            t.append(X[b * ell:(b + 1) * ell])
        out = []
        for v in t.complete_nodes():
            k, j = node_key(v)
            out.append((k, j + (index << (level - k)), v.H, v.V))
        return out


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def lazy_tree(wl, T):
    """An on-demand oracle tree over the first T slices of workload wl."""
    import synth
    from oracle.tree import LazyStreamSegmentTree
    t = LazyStreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol,
                              source=lambda a, b: synth.series(wl, a, b))
    t.append_blocks(T // wl.leaf_len)
    return t


def subtrees_under(tree, nodes, level):
    """Indices of the level-`level` subtrees lying under the given nodes (only
    nodes at or above that level count; smaller ones are left to the tree)."""
    from oracle.tree import node_key
    out = set()
    for v in nodes:
        k, j = node_key(v)
        if k >= level:
            out.update(range(j << (k - level), (j + 1) << (k - level)))
    return sorted(out)


def fill(tree, wl, level, indices, say=None):
    """Build the level-`level` subtrees `indices` in worker processes and store
    their nodes in `tree`."""
    todo = [i for i in indices if tree.node(level, i).H is None]
    if not todo:
        return 0
    ctx = mp.get_context("spawn")
    n = 0
    with ctx.Pool(min(workers(), len(todo))) as pool:
        for res in pool.imap_unordered(_subtree, [(wl.name, level, i) for i in todo]):
            for k, j, H, V in res:
                tree.put(k, j, H, V)
                n += 1
            if say:
                say("oracle subtree done (%d nodes so far)" % n)
    return n


def subtrees_for_ranges(tree, ranges, level):
    """Level-`level` subtrees under the hits of the given ranges (the hit
    sets come from the tree's structure; nothing is decomposed)."""
    from oracle.tree import StreamSegmentTree
    nodes = []
    for a, c in ranges:
        nodes += [v for v, _, _ in StreamSegmentTree.recall(tree, int(a), int(c))]
    return subtrees_under(tree, nodes, level)


def pool_level(wl, slices=256):
    """The subtree level whose nodes cover about `slices` slices."""
    return max(0, (max(1, slices // wl.leaf_len)).bit_length() - 1)
