"""Tucker-ALS (HOOI), effective ranks and the stopping rule.

Sec. 2: the optimal U^(n) with the other factors fixed is the r_n leading
left singular vectors of mat_n(X x_{m != n} U^(m)T) (Eq. "als-mat"); the
optimal core is X x_1 U^(1)T ... x_p U^(p)T.

Readings (the paper is silent on these):
  * initialisation: HOSVD, U^(n) = leading left singular vectors of mat_n(X);
  * stopping: fit_k = 1 - sqrt(max(0, |X|^2 - |G_k|^2)) / |X|; stop when
    |fit_k - fit_{k-1}| < tol (k >= 2) or k = max_iter (Sec. 8.1 gives
    "maximum 20 iterations, tolerance 0.01" without naming the quantity);
  * effective ranks: a factor with r orthonormal columns needs r <= its row
    count, and a mode rank can never exceed the product of the others, so
    ranks are clipped to r_1 <= length, r_n <= D_n, r_n <= prod_{m != n} r_m
    (iterated to a fixed point).
"""

from typing import List, Sequence, Tuple

import numpy as np

from .tensor_ops import fro2, mode_product, unfold


def effective_ranks(length: int, dims: Sequence[int], ranks: Sequence[int]) -> Tuple[int, ...]:
    """Clip the target ranks (r_1..r_p) to what a length x D_2 x ... x D_p tensor admits."""
    r = [min(int(ranks[0]), int(length))]
    r += [min(int(ranks[n]), int(dims[n - 1])) for n in range(1, len(ranks))]
    changed = True
    while changed:
        changed = False
        for n in range(len(r)):
            other = 1
            for m in range(len(r)):
                if m != n:
                    other *= r[m]
            if r[n] > other:
                r[n] = other
                changed = True
    return tuple(r)


def leading_left_singular_vectors(M: np.ndarray, k: int) -> np.ndarray:
    """The k leading left singular vectors of M (LAPACK SVD)."""
    U, _, _ = np.linalg.svd(M, full_matrices=False)
    return U[:, :k]


def fit_value(norm2_x: float, norm2_g: float) -> float:
    if norm2_x <= 0.0:
        return 1.0
    return 1.0 - np.sqrt(max(0.0, norm2_x - norm2_g)) / np.sqrt(norm2_x)


def converged(fits: List[float], tol: float) -> bool:
    return len(fits) >= 2 and abs(fits[-1] - fits[-2]) < tol


def hooi(X: np.ndarray, ranks: Sequence[int], max_iter: int = 20, tol: float = 0.01):
    """Tucker-ALS on an explicit tensor.

    Returns (G, [U^(1)..U^(p)], info) with info = {sweeps, fits, converged}.
    ``ranks`` are used as given (callers pass effective ranks).
    """
    p = X.ndim
    Us = [leading_left_singular_vectors(unfold(X, n), ranks[n]) for n in range(p)]
    nx = fro2(X)
    fits: List[float] = []
    G = None
    for _ in range(max_iter):
        for n in range(p):
            Y = X
            for m in range(p):
                if m != n:
                    Y = mode_product(Y, Us[m].T, m)
            Us[n] = leading_left_singular_vectors(unfold(Y, n), ranks[n])
        G = X
        for m in range(p):
            G = mode_product(G, Us[m].T, m)
        fits.append(fit_value(nx, fro2(G)))
        if converged(fits, tol):
            break
    if G is None:  # max_iter == 0: core of the HOSVD
        G = X
        for m in range(p):
            G = mode_product(G, Us[m].T, m)
    return G, Us, {"sweeps": len(fits), "fits": fits,
                   "converged": converged(fits, tol)}


def canonical_signs(G: np.ndarray, Us: List[np.ndarray]):
    """Flip factor columns so that each column's largest-magnitude entry is
    positive (lowest row on ties), flipping the matching core slices.  The
    represented tensor is unchanged."""
    G = G.copy()
    Us = [U.copy() for U in Us]
    for n, U in enumerate(Us):
        for j in range(U.shape[1]):
            i = int(np.argmax(np.abs(U[:, j])))
            if U[i, j] < 0:
                U[:, j] *= -1.0
                idx = [slice(None)] * G.ndim
                idx[n] = j
                G[tuple(idx)] *= -1.0
    return G, Us
