"""Shared helpers for the GPU parity tests (test-side only)."""

import sys
import time

import numpy as np

from oracle.evaluate import orthonormality_error, relative_error, subspace_sine
from oracle.tree import StreamSegmentTree


def say(*a):
    print("[gpu-test %.1fs]" % (time.time() % 1000), *a, flush=True)
    sys.stdout.flush()


def r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def oracle_tree(wl, X, T, max_iter=None, tol=None):
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta,
                          wl.max_iter if max_iter is None else max_iter,
                          wl.tol if tol is None else tol)
    for b in range(T // wl.leaf_len):
        t.append(X[b * wl.leaf_len:(b + 1) * wl.leaf_len])
    return t


def level_index(v):
    k = (v.hi - v.lo).bit_length() - 1
    return k, v.lo >> k


def round_nodes(orc):
    for v in orc.complete_nodes():
        v.H = r32(v.H)
        v.V = [r32(x) for x in v.V]


def load_store(gpu, orc):
    gpu.restore_begin(orc.T)
    for v in orc.complete_nodes():
        k, j = level_index(v)
        gpu.load_node(k, j, v.H, v.V)


def to_np(res):
    return res.core.double().cpu().numpy(), [u.double().cpu().numpy() for u in res.factors]


def leading_basis(G, Us, n, k):
    """First k left singular vectors of mat_n(G) mapped through U^(n): a
    gauge-free basis of the decomposition's leading mode-n subspace."""
    Gm = np.moveaxis(G, n, 0).reshape(G.shape[n], -1)
    W = np.linalg.svd(Gm, full_matrices=False)[0][:, :k]
    return Us[n] @ W


def gapped_rank(G, n, qmax, ratio=2.0):
    Gm = np.moveaxis(G, n, 0).reshape(G.shape[n], -1)
    s = np.linalg.svd(Gm, compute_uv=False)
    k = 0
    for i in range(1, min(qmax, len(s)) + 1):
        if i == len(s) or s[i - 1] >= ratio * s[i]:
            k = i
    return k


def compare(X, ts, te, G, U, Go, Uo, true_ranks=None, sine_tol=None):
    e_g = relative_error(X[ts:te], G, U)
    e_o = relative_error(X[ts:te], Go, Uo)
    delta = abs(e_g / e_o - 1.0) if e_o > 0 else abs(e_g)
    orth = max(orthonormality_error(u) for u in U)
    sine = 0.0
    if sine_tol is not None:
        for n in range(len(U)):
            qmax = U[n].shape[1] if true_ranks is None else min(U[n].shape[1], true_ranks[n])
            k = gapped_rank(Go, n, qmax)
            if k:
                sine = max(sine, subspace_sine(leading_basis(Go, Uo, n, k), leading_basis(G, U, n, k), k))
    return delta, orth, sine, e_g, e_o
