"""Evaluation helpers for the checks: errors, angles, brute force.

  * relative_error: |X - Y^|_F / |X|_F against the raw data, in FP64;
  * paper_metric: |X - Y_A| / |X - Y_ALS| - 1 (Sec. 8.1, "Evaluation
    metrics"), with Y_ALS from Tucker-ALS run from scratch on the range;
  * subspace_sine: sine of the largest principal angle between two column
    spans, |(I - A A^T) B|_2 for orthonormal A, B;
  * min_hitset_size: brute-force minimum of Eq. "prune-obj" subject to
    Eqs. "prune-c1" and "prune-c2", by dynamic programming over positions.
"""

from typing import Sequence

import numpy as np

from .tensor_ops import fro2, mode_product, tucker_to_tensor
from .tucker import effective_ranks, hooi


def reconstruct(G: np.ndarray, Us: Sequence[np.ndarray]) -> np.ndarray:
    return tucker_to_tensor(G, Us)


def relative_error(X: np.ndarray, G: np.ndarray, Us: Sequence[np.ndarray],
                   chunk: int = 4096) -> float:
    """|X - G x_1 U^(1) ... x_p U^(p)|_F / |X|_F, streamed over time."""
    num = 0.0
    den = 0.0
    U1 = np.asarray(Us[0], dtype=np.float64)
    rest = [np.asarray(U, dtype=np.float64) for U in Us[1:]]
    Gd = np.asarray(G, dtype=np.float64)
    for t0 in range(0, X.shape[0], chunk):
        t1 = min(X.shape[0], t0 + chunk)
        Y = mode_product(Gd, U1[t0:t1], 0)
        for n, U in enumerate(rest, start=1):
            Y = mode_product(Y, U, n)
        D = np.asarray(X[t0:t1], dtype=np.float64) - Y
        num += fro2(D)
        den += fro2(X[t0:t1])
    return float(np.sqrt(num / den)) if den > 0 else 0.0


def paper_metric(X: np.ndarray, G: np.ndarray, Us, ranks: Sequence[int],
                 max_iter: int = 20, tol: float = 0.01) -> float:
    Gb, Ub, _ = hooi(np.asarray(X, dtype=np.float64), ranks, max_iter, tol)
    e_als = relative_error(X, Gb, Ub)
    e_a = relative_error(X, G, Us)
    return e_a / e_als - 1.0 if e_als > 0 else 0.0


def subspace_sine(A: np.ndarray, B: np.ndarray, k: int) -> float:
    """sin of the largest principal angle between span(A[:, :k]) and span(B[:, :k])."""
    A = np.asarray(A, dtype=np.float64)[:, :k]
    B = np.asarray(B, dtype=np.float64)[:, :k]
    Qa = np.linalg.qr(A)[0]
    Qb = np.linalg.qr(B)[0]
    R = Qb - Qa @ (Qa.T @ Qb)
    if R.size == 0:
        return 0.0
    return float(min(1.0, np.linalg.norm(R, 2)))


def orthonormality_error(U: np.ndarray) -> float:
    U = np.asarray(U, dtype=np.float64)
    return float(np.max(np.abs(U.T @ U - np.eye(U.shape[1])))) if U.size else 0.0


def min_hitset_size(tree, ts: int, te: int) -> int:
    """Smallest S of complete nodes whose clipped ranges partition [ts, te)
    and each meet the threshold (leaves always allowed, they are terminal)."""
    num, den = tree.theta
    cand = []
    for v in tree.complete_nodes():
        s, t = tree.sigma(v), tree.tau(v)
        lo, hi = max(ts, s), min(te, t)
        if hi <= lo:
            continue
        if v.kind == "L" or den * (hi - lo) >= num * (t - s):
            cand.append((lo, hi))
    INF = 1 << 30
    best = {ts: 0}
    for x in range(ts, te):
        if x not in best:
            continue
        for lo, hi in cand:
            if lo == x and best.get(hi, INF) > best[x] + 1:
                best[hi] = best[x] + 1
    return best.get(te, INF)


def tucker_ranks_for(length: int, dims, ranks):
    return effective_ranks(length, dims, ranks)
