"""Pins for the oracle's stream segment tree and Recall (structure only).

Checked against the paper's worked example (Fig. "illust"), the height
theorem (Thm. "alg-log-height"), the hit-set bound (Lemma "hit-height"),
the optimality/visit bounds of Alg. "recall" (Thm. "prune-opt" and its
proof), the amortized merge count (Prop. "time_complexity_appending"), and a
brute-force minimum of Eq. "prune-obj".
"""

import math
import os

import numpy as np
import pytest

from oracle.evaluate import min_hitset_size
from oracle.tree import StreamSegmentTree

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "illust_tree.txt")


def _structure_tree(T_b, leaf_len=1, theta=(7, 10)):
    t = StreamSegmentTree(dims=(2, 2), ranks=(1, 1, 1), leaf_len=leaf_len, theta=theta)
    for _ in range(T_b):
        t.append(None)
    return t


def _golden():
    nodes, hits, rec = {}, [], None
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "recall":
                rec = tuple(int(x) for x in line[1:])
            elif line[0] == "hit":
                hits.append(tuple(int(x) for x in line[1:]))
            else:
                nodes[int(line[0])] = (int(line[1]), int(line[2]), line[3])
    return nodes, rec, hits


def test_paper_example_tree():
    nodes, _, _ = _golden()
    t = _structure_tree(9)
    got = {v.id: (t.sigma(v), t.tau(v), v.kind) for v in t.nodes}
    assert got == nodes
    assert t.height() == 5 == math.ceil(math.log2(9)) + 1
    leaves = [v.id for v in sorted(t.nodes, key=lambda v: v.lo) if v.kind == "L"]
    assert leaves == [1, 3, 6, 7, 11, 12, 14, 15, 20]
    assert t.root.id == 16 and t.root.left.id == 8 and t.root.right.id == 17


def test_paper_example_recall():
    _, rec, hits = _golden()
    ts, te, num, den = rec
    t = _structure_tree(9, theta=(num, den))
    got = [(v.id, lo, hi, int(not (lo == t.sigma(v) and hi == t.tau(v))))
           for v, lo, hi in t.recall(ts, te)]
    assert got == hits


@pytest.mark.parametrize("T_b", list(range(1, 130)) + [255, 256, 257, 511, 512, 513, 1000])
def test_height_theorem(T_b):
    t = _structure_tree(T_b)
    expect = 1 if T_b == 1 else math.ceil(math.log2(T_b)) + 1
    assert t.height() == expect


def _trailing_ones(b):
    n = 0
    while b & 1:
        n += 1
        b >>= 1
    return n


def test_merges_per_append_and_node_count():
    t = StreamSegmentTree(dims=(2, 2), ranks=(1, 1, 1))
    for b in range(700):
        t.append(None)
        assert t.merges_last == _trailing_ones(b)
        T_b = b + 1
        assert t.merges_total == T_b - bin(T_b).count("1")
        K = 0 if T_b == 1 else math.ceil(math.log2(T_b))
        assert len(t.nodes) == sum(-(-T_b // (1 << k)) for k in range(K + 1))
        # worst case is floor(log2(b+1)) merges, amortised below one
        assert t.merges_last <= int(math.log2(b + 1))


def _closed_form_ids(T_b):
    """Creation order of dyadic node (k, j): created at block c = 2^(k-1) if
    j = 0 and k >= 1, else c = j 2^k; blocks before c create
    [c>=1] + [c>=2](2(c-1) - popcount(c-1) + bitlen(c-1)) nodes; at c the new
    root (bitlen(c), 0) comes first when c is a power of two, then
    (k', c >> k') for k' = nu_2(c) down to 0."""
    def before(c):
        if c == 0:
            return 0
        if c == 1:
            return 1
        m = c - 1
        return 1 + 2 * m - bin(m).count("1") + m.bit_length()

    ids = {}
    for c in range(T_b):
        order = []
        if c == 0:
            order = [(0, 0)]
        else:
            if c & (c - 1) == 0:
                order.append((c.bit_length(), 0))
            nu = (c & -c).bit_length() - 1
            for k in range(nu, -1, -1):
                order.append((k, c >> k))
        for pos, kj in enumerate(order):
            ids[kj] = before(c) + 1 + pos
    return ids


def test_closed_form_ids():
    T_b = 600
    t = _structure_tree(T_b)
    ids = _closed_form_ids(T_b)
    for v in t.nodes:
        k = (v.hi - v.lo).bit_length() - 1
        assert (v.hi - v.lo) == 1 << k and v.lo % (1 << k) == 0   # dyadic
        assert ids[(k, v.lo >> k)] == v.id


@pytest.mark.parametrize("theta", [(1, 2), (7, 10), (9, 10), (1, 1)])
@pytest.mark.parametrize("leaf_len", [1, 3])
def test_recall_optimal_and_bounded(theta, leaf_len):
    for T_b in list(range(1, 24)) + [37]:
        t = _structure_tree(T_b, leaf_len=leaf_len, theta=theta)
        h = t.height()
        T = t.T
        for ts in range(T):
            for te in range(ts + 1, T + 1):
                visited = []
                hits = t.recall(ts, te, visited)
                # clipped ranges partition [ts, te) in time order (Eq. "prune-c1")
                assert hits[0][1] == ts and hits[-1][2] == te
                for a, b in zip(hits, hits[1:]):
                    assert a[2] == b[1]
                # threshold (Eq. "prune-c2"); leaves are terminal
                for v, lo, hi in hits:
                    assert v.kind in ("L", "M")
                    if v.kind == "M":
                        assert theta[1] * (hi - lo) >= theta[0] * (t.tau(v) - t.sigma(v))
                partial = sum(1 for v, lo, hi in hits
                              if not (lo == t.sigma(v) and hi == t.tau(v)))
                assert partial <= 2
                assert len(hits) <= max(2 * (h - 1), 1)
                assert len(visited) <= 4 * h - 2
                assert len(hits) == min_hitset_size(t, ts, te)


def test_recall_rejects_out_of_range():
    t = _structure_tree(5, leaf_len=2)
    for ts, te in [(0, 0), (3, 2), (-1, 2), (0, 11)]:
        with pytest.raises(ValueError):
            t.recall(ts, te)


# --- the fixed-block hit set (the flat partition of the efficiency-accuracy comparison) ---

def test_fixed_block_hits_worked_examples():
    """Worked by hand.  64 blocks of one slice, level 2 (blocks of 4): the
    range [5, 19) takes [4,8) clipped to [5,8), [8,12), [12,16) and [16,20)
    clipped to [16,19).  22 blocks, level 3 (blocks of 8): only [0,8) and
    [8,16) are complete, so [3, 21) takes [3,8), [8,16) and then Alg.
    "recall" on [16, 21): the node [16,20) and the leaf [20,21)."""
    t = _structure_tree(64)
    got = [(t.sigma(v), t.tau(v), lo, hi) for v, lo, hi in t.fixed_block_hits(5, 19, 2)]
    assert got == [(4, 8, 5, 8), (8, 12, 8, 12), (12, 16, 12, 16), (16, 20, 16, 19)]
    t = _structure_tree(22)
    got = [(t.sigma(v), t.tau(v), lo, hi) for v, lo, hi in t.fixed_block_hits(3, 21, 3)]
    assert got == [(0, 8, 3, 8), (8, 16, 8, 16), (16, 20, 16, 20), (20, 21, 20, 21)]


@pytest.mark.parametrize("T_b,leaf_len,level", [(100, 1, 3), (37, 4, 2), (256, 2, 5), (9, 1, 0)])
def test_fixed_block_hits_tile_the_range(T_b, leaf_len, level):
    """Every range: the hits tile it in time order, each is clipped to its
    node, and all hits before the last complete block boundary are nodes of
    the chosen level."""
    t = _structure_tree(T_b, leaf_len=leaf_len)
    T = T_b * leaf_len
    B = leaf_len << level
    full_end = (T_b >> level) * B
    rng = np.random.default_rng(T_b + level)
    for _ in range(200):
        ts, te = sorted(rng.choice(T + 1, size=2, replace=False).tolist())
        hits = t.fixed_block_hits(ts, te, level)
        pos = ts
        for v, lo, hi in hits:
            assert lo == pos and lo < hi and t.sigma(v) <= lo and hi <= t.tau(v)
            if hi <= full_end:
                assert t.tau(v) - t.sigma(v) == B
            else:
                assert lo >= full_end
            pos = hi
        assert pos == te
