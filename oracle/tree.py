"""Stream segment tree with Alg. "append", Alg. "insert" and Alg. "recall".

Sec. 4.2 defines leaf (L), intermediate (M) and placeholder (P) nodes; Sec.
6.2 gives the append/insert procedures; Sec. 5.1 gives the pruned hit set.

Readings:
  * leaves hold blocks of ``leaf_len`` slices (the paper's leaf is one slice,
    leaf_len = 1); the tree algorithms run on block indices and node ranges
    are reported in slices.  Only whole blocks are committed, so queries need
    te <= T_c = leaf_len * (number of complete blocks);
  * a leaf reached by Recall is accepted even below the threshold (it has no
    children) and is trimmed like a partial hit;
  * theta = num/den and the test |[ts,te) & [s,t)| >= theta |[s,t)| is done
    in integers as den * overlap >= num * length;
  * node ids are the 1-based creation order, which reproduces the numbering of
    the paper's example (Fig. "illust");
  * the new root made by Alg. "append" is a placeholder whose range is
    [0, 2 tau_r) and whose left child is the old root (the prose has typos);
  * a range equal to one node returns that node's stored decomposition;
    every other query goes through Alg. "stitch".
"""

from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import stitch as stitch_mod
from .tucker import canonical_signs, effective_ranks, hooi


class Node:
    __slots__ = ("id", "lo", "hi", "kind", "left", "right", "H", "V", "info")

    def __init__(self, nid: int, lo: int, hi: int):
        self.id = nid          # creation order, 1-based
        self.lo = lo           # range in blocks [lo, hi)
        self.hi = hi
        self.kind = "P"
        self.left: Optional["Node"] = None
        self.right: Optional["Node"] = None
        self.H = None
        self.V = None
        self.info = None


class StreamSegmentTree:
    """Literal pointer-based stream segment tree over blocks of slices.

    ``append(block)`` takes a leaf_len x D_2 x ... x D_p array (or None for a
    structure-only tree, which skips every decomposition).
    """

    def __init__(self, dims: Sequence[int], ranks: Sequence[int], leaf_len: int = 1,
                 theta: Tuple[int, int] = (7, 10), max_iter: int = 20, tol: float = 0.01):
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.leaf_len = int(leaf_len)
        self.theta = (int(theta[0]), int(theta[1]))
        self.max_iter = int(max_iter)
        self.tol = float(tol)
        self.root: Optional[Node] = None
        self.T_b = 0                 # committed blocks
        self.next_id = 1
        self.nodes: List[Node] = []  # in creation order
        self.merges_last = 0         # stitches run by the last append
        self.merges_total = 0

    # -- helpers ------------------------------------------------------------
    @property
    def T(self) -> int:
        """Committed timespan in slices."""
        return self.T_b * self.leaf_len

    def sigma(self, v: Node) -> int:
        return v.lo * self.leaf_len

    def tau(self, v: Node) -> int:
        return v.hi * self.leaf_len

    def _new(self, lo: int, hi: int) -> Node:
        v = Node(self.next_id, lo, hi)
        self.next_id += 1
        self.nodes.append(v)
        return v

    def height(self) -> int:
        def h(v):
            if v is None:
                return 0
            return 1 + max(h(v.left), h(v.right))
        return h(self.root)

    # -- Alg. "append" and Alg. "insert" (Sec. 6.2) ----------------------------
    # The stream segment tree is a dyadic tree over block indices grown on
    # demand.  Appending block T (a) doubles the root when T reaches its end
    # (the new root is a placeholder [0, 2 tau) with the old root on its left),
    # (b) walks from the root to the slot [T, T+1), creating the missing
    # placeholders on the way (in that order, which fixes the node ids), (c)
    # turns the slot into a leaf holding the block's Tucker decomposition, and
    # (d) finishes, from the bottom up, every node on that path whose range now
    # ends at T+1: each becomes an intermediate node whose decomposition is
    # the Stitch of its two children.
    def append(self, block: Optional[np.ndarray]) -> None:
        T = self.T_b
        if self.root is None:
            self.root = self._new(0, 1)
        elif T == self.root.hi:
            grown = self._new(0, 2 * self.root.hi)
            grown.left = self.root
            self.root = grown
        path = [self.root]
        while path[-1].hi - path[-1].lo > 1:
            v = path[-1]
            half = (v.lo + v.hi) // 2
            side = "left" if T < half else "right"
            child = getattr(v, side)
            if child is None:
                child = self._new(v.lo, half) if side == "left" else self._new(half, v.hi)
                setattr(v, side, child)
            path.append(child)
        leaf = path[-1]
        assert leaf.lo == T, "the walk must end at the new block's slot"
        leaf.kind = "L"
        if block is not None:
            self._decompose_leaf(leaf, block)
        self.merges_last = 0
        for v in reversed(path[:-1]):
            if v.hi != T + 1:
                break  # nodes above end later; none of them completes now
            self._complete(v, block is not None)
        self.T_b += 1
        self.merges_total += self.merges_last

    def _complete(self, v: Node, decompose: bool) -> None:
        """v's last block has arrived: it becomes intermediate, stitched from
        its children at the ranks its length admits."""
        v.kind = "M"
        self.merges_last += 1
        if decompose:
            self._decompose_merge(v)

    def _decompose_leaf(self, leaf: Node, block: np.ndarray) -> None:
        """A leaf holds the Tucker-ALS decomposition of its raw block."""
        r = effective_ranks(self.leaf_len, self.dims, self.ranks)
        G, U, info = hooi(np.asarray(block, dtype=np.float64), r, self.max_iter, self.tol)
        leaf.H, leaf.V = canonical_signs(G, U)
        leaf.info = info

    def _decompose_merge(self, v: Node) -> None:
        """A completed intermediate node holds the Stitch of its two children."""
        r = effective_ranks((v.hi - v.lo) * self.leaf_len, self.dims, self.ranks)
        pieces = [stitch_mod.Piece(v.left.H, v.left.V), stitch_mod.Piece(v.right.H, v.right.V)]
        v.H, v.V, v.info = stitch_mod.stitch(pieces, r, self.max_iter, self.tol)

    # -- Alg. "recall" (Sec. 5.1) ---------------------------------------------
    def _accept(self, v: Node, ts: int, te: int) -> bool:
        inter = max(0, min(te, self.tau(v)) - max(ts, self.sigma(v)))
        num, den = self.theta
        return den * inter >= num * (self.tau(v) - self.sigma(v))

    def recall(self, ts: int, te: int, _visited: Optional[list] = None) -> List[Tuple[Node, int, int]]:
        """Pruned hit set of [ts, te) in time order: (node, lo, hi) with the
        clipped range [lo, hi) in slices.  Starting from the root, a node is
        taken whole when it is complete and the range covers at least theta of
        it, or when it is a leaf (nothing below it to refine); any other node
        hands the search to those of its children that overlap the range,
        earlier child first."""
        if not (0 <= ts < te <= self.T):
            raise ValueError("range [%d,%d) not inside [0,%d)" % (ts, te, self.T))
        out: List[Node] = []
        todo = [self.root]
        while todo:
            v = todo.pop()
            if _visited is not None:
                _visited.append(v)
            if v.kind == "L" or (v.kind == "M" and self._accept(v, ts, te)):
                out.append(v)
                continue
            kids = [u for u in (v.left, v.right)
                    if u is not None and max(ts, self.sigma(u)) < min(te, self.tau(u))]
            assert kids, "a node inside the range without children"
            todo.extend(reversed(kids))  # the earlier child is popped first
        return [(v, max(ts, self.sigma(v)), min(te, self.tau(v))) for v in out]

    def fixed_block_hits(self, ts: int, te: int, level: int) -> List[Tuple[Node, int, int]]:
        """The fixed-block variant of the hit set (the flat partition the
        paper compares against): every complete node of `level` (blocks of
        leaf_len 2^level slices) that overlaps [ts, te), clipped to it; the
        part of the range past the last complete node of that level (less
        than one block, near the committed end) comes from Alg. "recall" on
        that remainder.  In time order, tiling [ts, te)."""
        if not (0 <= ts < te <= self.T):
            raise ValueError("range [%d,%d) not inside [0,%d)" % (ts, te, self.T))
        B = self.leaf_len << level
        full_end = (self.T_b >> level) * B
        level_nodes = {}
        for v in self.complete_nodes():
            if v.hi - v.lo == (1 << level):
                level_nodes[v.lo >> level] = v
        out = []
        j = ts // B
        while j * B < min(te, full_end):
            v = level_nodes[j]
            out.append((v, max(ts, j * B), min(te, (j + 1) * B)))
            j += 1
        if te > full_end:
            out += self.recall(max(ts, full_end), te)
        return out

    # -- Sec. 6.1 query ----------------------------------------------------------
    def provisional_piece(self, tail):
        """The decomposition of an incomplete block (1 <= m < leaf_len slices
        appended past the last complete block): the leaf procedure (Tucker-ALS,
        node ranks clipped to length m) on those slices; nothing is stored."""
        X = np.asarray(tail, dtype=np.float64)
        if not (1 <= X.shape[0] < self.leaf_len):
            raise ValueError("a tail has 1 .. leaf_len-1 slices")
        r = effective_ranks(X.shape[0], self.dims, self.ranks)
        G, U, _ = hooi(X, r, self.max_iter, self.tol)
        return canonical_signs(G, U)

    def query(self, ts: int, te: int, max_iter: Optional[int] = None,
              tol: Optional[float] = None, ranks: Optional[Sequence[int]] = None,
              level: Optional[int] = None, tail=None):
        """Tucker decomposition of X[ts:te): Recall, trims, Stitch.
        ranks: output ranks r_1..r_p, each at most the tree's (default: the
        tree's); Alg. "stitch" takes the target ranks as an input, so a query
        may ask for less than the nodes hold.  A range equal to one stored
        node is returned verbatim only at the node's own ranks.  level: the
        fixed-block hit set of that level instead of Alg. "recall".  tail:
        the slices appended past the last complete block; a range reaching
        into them takes the provisional piece of that block, trimmed like a
        partial hit, after the hits of its committed part.
        Returns (G, [U^(1)..U^(p)], info)."""
        max_iter = self.max_iter if max_iter is None else max_iter
        tol = self.tol if tol is None else tol
        req = self.ranks if ranks is None else tuple(int(x) for x in ranks)
        if len(req) != len(self.ranks) or any(not (1 <= x <= R) for x, R in zip(req, self.ranks)):
            raise ValueError("query ranks must be in [1, node rank] per mode")
        r = effective_ranks(te - ts, self.dims, req)
        Tc = self.T
        m = 0 if tail is None else len(tail)
        if not (0 <= ts < te <= Tc + m):
            raise ValueError("range [%d,%d) not inside [0,%d)" % (ts, te, Tc + m))
        tec = min(te, Tc)
        hits = []
        if ts < tec:
            hits = self.recall(ts, tec) if level is None else self.fixed_block_hits(ts, tec, level)
        if te > Tc:
            H, V = self.provisional_piece(tail)
            lo = max(ts, Tc)
            G, U, info = stitch_mod.stitch(
                [self._piece(v, a, b) for v, a, b in hits] + [stitch_mod.trim(H, V, lo - Tc, te - lo)],
                r, max_iter, tol)
            info["hits"] = hits
            info["tail"] = (lo, te)
            return G, U, info
        if len(hits) == 1 and hits[0][1] == self.sigma(hits[0][0]) and hits[0][2] == self.tau(hits[0][0]) \
                and r == tuple(hits[0][0].H.shape):
            v = hits[0][0]
            return v.H.copy(), [U.copy() for U in v.V], {
                "sweeps": 0, "fits": [], "converged": True, "hits": hits,
                "err_model": None, "norm_ytilde": None}
        G, U, info = stitch_mod.stitch([self._piece(v, lo, hi) for v, lo, hi in hits], r, max_iter, tol)
        info["hits"] = hits
        return G, U, info

    def _piece(self, v: Node, lo: int, hi: int):
        """A hit as a piece: the node itself, or its trim to [lo, hi)."""
        if lo == self.sigma(v) and hi == self.tau(v):
            return stitch_mod.Piece(v.H, list(v.V))
        return stitch_mod.trim(v.H, v.V, lo - self.sigma(v), hi - lo)

    def pieces(self, ts: int, te: int):
        """The pieces Y~_i of a query (after trims), for the checks."""
        out = []
        for v, lo, hi in self.recall(ts, te):
            if lo == self.sigma(v) and hi == self.tau(v):
                out.append(stitch_mod.Piece(v.H, list(v.V)))
            else:
                out.append(stitch_mod.trim(v.H, v.V, lo - self.sigma(v), hi - lo))
        return out

    def complete_nodes(self) -> List[Node]:
        return [v for v in self.nodes if v.kind in ("L", "M")]


def node_key(v: Node) -> Tuple[int, int]:
    """(level, index) of a complete node: level k holds nodes of 2^k blocks,
    index j covers blocks [j 2^k, (j+1) 2^k)."""
    k = (v.hi - v.lo).bit_length() - 1
    return k, v.lo >> k


class LazyStreamSegmentTree(StreamSegmentTree):
    """The same tree with every decomposition made on first use.

    ``append_blocks(n)`` grows the structure only; ``source(t0, t1)`` returns
    the raw slices [t0, t1).  A node's decomposition depends on nothing but
    the slices under it (a leaf is Tucker-ALS of its block, an intermediate
    node the Stitch of its children), so computing it when a query first
    needs it, from the bottom of its subtree up, gives exactly what the eager
    tree holds.  ``put(level, index, H, V)`` stores a decomposition computed
    elsewhere by this package (for example by an eager tree over the same
    slices); ``ensure`` makes one on demand.
    """

    def __init__(self, dims, ranks, leaf_len=1, theta=(7, 10), max_iter=20, tol=0.01, source=None):
        super().__init__(dims, ranks, leaf_len, theta, max_iter, tol)
        self.source = source
        self._by_key = {}

    def append_blocks(self, n: int) -> None:
        for _ in range(int(n)):
            self.append(None)

    def _index(self):
        if len(self._by_key) != len(self.nodes):
            self._by_key = {node_key(v): v for v in self.complete_nodes()}
        return self._by_key

    def node(self, level: int, index: int) -> Node:
        return self._index()[(int(level), int(index))]

    def put(self, level: int, index: int, H, V) -> None:
        v = self.node(level, index)
        v.H, v.V = H, list(V)

    def ensure(self, v: Node) -> None:
        if v.H is not None:
            return
        if v.kind == "L":
            ell = self.leaf_len
            self._decompose_leaf(v, self.source(v.lo * ell, v.hi * ell))
            return
        assert v.kind == "M", "only complete nodes hold decompositions"
        self.ensure(v.left)
        self.ensure(v.right)
        self._decompose_merge(v)

    def recall(self, ts, te, _visited=None):
        hits = super().recall(ts, te, _visited)
        for v, _, _ in hits:
            self.ensure(v)
        return hits

    def fixed_block_hits(self, ts, te, level):
        hits = super().fixed_block_hits(ts, te, level)
        for v, _, _ in hits:
            self.ensure(v)
        return hits
