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


def data_spectrum(X, Uo, n):
    """Singular values of mat_n(X x_{m != n} U_o^(m)T): the first r_n are
    those of the oracle's core (at an ALS fixed point), the rest show the
    gap at the rank cut, which the core alone cannot."""
    Y = np.asarray(X, dtype=np.float64)
    for m, U in enumerate(Uo):
        if m != n:
            Y = np.moveaxis(np.tensordot(np.asarray(U, dtype=np.float64).T, Y, axes=(1, m)), 0, m)
    Ym = np.moveaxis(Y, n, 0).reshape(Y.shape[n], -1)
    return np.linalg.svd(Ym, compute_uv=False)


# Unit roundoff of FP32: the device's contractions perturb each Gram by
# about U32 times its largest eigenvalue (FP32 operands and products, FP64
# Gram sums), so by Davis-Kahan the leading-k subspace of a mode may turn by
# up to about U32 s_1^2 / (s_k^2 - s_{k+1}^2).
U32 = 2.0 ** -24
GRAM_ROUNDING = 1.0


def gapped_rank_of(s, qmax, ratio=2.0, resolvable=None):
    """Largest k <= qmax with s[k-1] >= ratio s[k] (k = len(s): no next
    value).  With resolvable=b, also require the Davis-Kahan bound of the
    leading-k subspace under FP32 rounding of the Gram,
    GRAM_ROUNDING U32 s_1^2 / (s_k^2 - s_{k+1}^2), to be at most b: the
    directions FP32 contractions can determine to that accuracy."""
    k = 0
    for i in range(1, min(qmax, len(s)) + 1):
        if i == len(s) or s[i - 1] >= ratio * s[i]:
            if resolvable is not None and i < len(s):
                gap = s[i - 1] ** 2 - s[i] ** 2
                if not (gap > 0 and GRAM_ROUNDING * U32 * s[0] ** 2 / gap <= resolvable):
                    continue
            k = i
    return k


def ytilde(orc, ts, te):
    """The oracle's stitched tensor Y~ of [ts, te): its pieces (hits after
    trims) materialised and concatenated along time."""
    from oracle.evaluate import reconstruct
    return np.concatenate([reconstruct(pc.H, pc.V) for pc in orc.pieces(ts, te)], axis=0)


EXACT = 1e-5  # an oracle error below this is FP32-level: the gate is the device's own error


def node_delta(e_g, e_o):
    """The error-ratio gap |e_gpu / e_oracle - 1|; where the oracle's
    decomposition is exact to below FP32 resolution (a node whose ranks
    reach its shape), the ratio has no meaning and the device's own
    relative error is gated instead."""
    return abs(e_g / e_o - 1.0) if e_o > EXACT else abs(e_g)


def compare(X, ts, te, G, U, Go, Uo, true_ranks=None, sine_tol=None, Yt=None):
    """Error ratio, orthonormality and (with sine_tol) the largest sine
    between the leading subspaces of each mode, over the directions up to
    the generator's rank that the stitched tensor's projected spectrum
    (Yt = Y~, else the raw range) separates from the next one by a factor
    of 2, and whose Davis-Kahan bound under FP32 rounding is within
    sine_tol."""
    e_g = relative_error(X[ts:te], G, U)
    e_o = relative_error(X[ts:te], Go, Uo)
    delta = node_delta(e_g, e_o)
    orth = max(orthonormality_error(u) for u in U)
    sine = 0.0
    if sine_tol is not None:
        Ys = X[ts:te] if Yt is None else Yt
        for n in range(len(U)):
            qmax = U[n].shape[1] if true_ranks is None else min(U[n].shape[1], true_ranks[n])
            k = gapped_rank_of(data_spectrum(Ys, Uo, n), qmax, resolvable=sine_tol)
            if k:
                sine = max(sine, subspace_sine(leading_basis(Go, Uo, n, k), leading_basis(G, U, n, k), k))
    return delta, orth, sine, e_g, e_o


def recon_diff(G, U, Go, Uo):
    """|Y^_gpu - Y^_oracle|_F / |Y^_oracle|_F, the two reconstructions
    G x_1 U^(1) ... x_p U^(p) formed in FP64."""
    from oracle.evaluate import reconstruct
    Yg = reconstruct(np.asarray(G, dtype=np.float64), [np.asarray(u, dtype=np.float64) for u in U])
    Yo = reconstruct(np.asarray(Go, dtype=np.float64), [np.asarray(u, dtype=np.float64) for u in Uo])
    return float(np.linalg.norm((Yg - Yo).ravel()) / max(1e-300, np.linalg.norm(Yo.ravel())))


def recon_bound(Yt, Go, Uo):
    """Davis-Kahan estimate of how far FP32 rounding may move a converged
    reconstruction, relative to its norm: per mode, the subspace at the rank
    cut turns by about U32 s_1^2 / (s_r^2 - s_{r+1}^2) and carries energy
    about s_r (spectrum of the stitched tensor Y~ projected on the oracle's
    other factors); summed over modes.  Infinite when a cut has no gap."""
    tot = 0.0
    for n in range(len(Uo)):
        s = data_spectrum(Yt, Uo, n)
        r = Uo[n].shape[1]
        if r < len(s):
            gap = s[r - 1] ** 2 - s[r] ** 2
            if not gap > 0:
                return float("inf")
            tot += U32 * s[0] ** 2 * s[r - 1] / gap
    return tot / max(1e-300, float(np.linalg.norm(np.asarray(Go).ravel())))
