"""Partial-hit approximation and Alg. "stitch" (Sec. 5), literal FP64 form.

A piece Y~_i = H~_i x_1 V~_i^(1) ... x_p V~_i^(p) is given by its core and
factors; Y~ is the concatenation of the pieces along the temporal mode.

Readings (where the paper is silent or garbled):
  * row offsets t_i use the clipped length of each hit (the number of rows of
    V~_i^(1)); with the full node length, as Alg. "stitch" prints it, the row
    blocks would not add up to the query length;
  * Alg. "stitch" initialises U^(2..p) at random; here they are the HOSVD of
    Y~, i.e. the leading eigenvectors of the exact Gram mat_n(Y~) mat_n(Y~)T,
    formed from the pieces without materialising Y~;
  * "until converged" uses the fit rule of ``tucker.hooi`` with
    |Y~|^2 computed exactly from the pieces;
  * the garbled Eq. "stitch-temp-1" is read as Y~ x_2 U^(2)T ... x_p U^(p)T.
"""

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from .tensor_ops import fold, fro2, mode_product, unfold
from .tucker import canonical_signs, converged, fit_value, leading_left_singular_vectors


@dataclass
class Piece:
    H: np.ndarray            # core, k x r_2 x ... x r_p
    V: List[np.ndarray]      # [V^(1) (rows x k), V^(2) (D_2 x r_2), ...]


def trim(H: np.ndarray, V: List[np.ndarray], a: int, l: int) -> Piece:
    """Eq. "partial-tucker": rows [a, a+l) of V^(1) = Q~ R~ (reduced QR);
    the piece is (H x_1 R~, [Q~, V^(2), ...])."""
    Q, R = np.linalg.qr(V[0][a:a + l], mode="reduced")
    return Piece(mode_product(H, R, 0), [Q] + list(V[1:]))


def ytilde_norm2(pieces: Sequence[Piece]) -> float:
    """|Y~|^2 = sum_i <H_i, H_i x_1 Gamma_1 ... x_p Gamma_p>, Gamma_n = V^(n)T V^(n)
    (exact even when the factors are not perfectly orthonormal)."""
    total = 0.0
    for pc in pieces:
        T = pc.H
        for n, V in enumerate(pc.V):
            T = mode_product(T, V.T @ V, n)
        total += float(np.sum(pc.H * T))
    return total


def _gram_hosvd(pieces: Sequence[Piece], n: int) -> np.ndarray:
    """mat_n(Y~) mat_n(Y~)T for a non-temporal mode n, from the pieces:
    sum_i V_n mat_n(H_i) (kron_{m != n} V_m^T V_m) mat_n(H_i)^T V_n^T."""
    D = pieces[0].V[n].shape[0]
    S = np.zeros((D, D))
    for pc in pieces:
        T = pc.H
        for m, V in enumerate(pc.V):
            if m != n:
                T = mode_product(T, V.T @ V, m)
        C = unfold(T, n) @ unfold(pc.H, n).T
        S += pc.V[n] @ C @ pc.V[n].T
    return 0.5 * (S + S.T)


def _top_eigvecs(S: np.ndarray, k: int) -> np.ndarray:
    w, E = np.linalg.eigh(S)
    order = np.argsort(-w, kind="stable")
    return E[:, order[:k]]


def stitch(pieces: Sequence[Piece], ranks: Sequence[int], max_iter: int = 20,
           tol: float = 0.01):
    """Alg. "stitch": Tucker-ALS of the virtual concatenation Y~.

    Z^(1) is built explicitly as an L x prod(r_2..r_p) matrix, block i being
    V~_i^(1) mat_1(H~_i x_2 (U^(2)T V~_i^(2)) ... x_p (U^(p)T V~_i^(p)))
    (Eq. "stitch-temp-2"); Z^(n), n >= 2, follows Eq. "stitch-nontemp-3".
    Returns (G, [U^(1)..U^(p)], info) with canonical signs applied.
    """
    p = len(pieces[0].V)
    rows = [pc.V[0].shape[0] for pc in pieces]
    t = np.concatenate([[0], np.cumsum(rows)]).astype(int)
    U: List[np.ndarray] = [None] * p
    for n in range(1, p):
        U[n] = _top_eigvecs(_gram_hosvd(pieces, n), ranks[n])
    ny = ytilde_norm2(pieces)
    fits: List[float] = []
    G = None
    for _ in range(max_iter):
        # temporal mode (Eq. "stitch-temp-2")
        blocks = []
        for pc in pieces:
            W = pc.H
            for m in range(1, p):
                W = mode_product(W, U[m].T @ pc.V[m], m)
            blocks.append(pc.V[0] @ unfold(W, 0))
        Z1 = np.vstack(blocks)
        U[0] = leading_left_singular_vectors(Z1, ranks[0])
        # non-temporal modes (Eq. "stitch-nontemp-3")
        Zn = None
        for n in range(1, p):
            Zn = None
            for i, pc in enumerate(pieces):
                W = mode_product(pc.H, U[0][t[i]:t[i + 1]].T @ pc.V[0], 0)
                for m in range(1, p):
                    if m != n:
                        W = mode_product(W, U[m].T @ pc.V[m], m)
                W = mode_product(W, pc.V[n], n)
                term = unfold(W, n)
                Zn = term if Zn is None else Zn + term
            U[n] = leading_left_singular_vectors(Zn, ranks[n])
        # core update: reshape Z^(p) and multiply by U^(p)T
        shape = [ranks[m] for m in range(p - 1)] + [U[p - 1].shape[0]]
        G = mode_product(fold(Zn, p - 1, shape), U[p - 1].T, p - 1)
        fits.append(fit_value(ny, fro2(G)))
        if converged(fits, tol):
            break
    G, U = canonical_signs(G, U)
    err = np.sqrt(max(0.0, ny - fro2(G))) / np.sqrt(ny) if ny > 0 else 0.0
    return G, U, {"sweeps": len(fits), "fits": fits, "converged": converged(fits, tol),
                  "err_model": float(err), "norm_ytilde": float(np.sqrt(ny))}


def z_matrices(pieces: Sequence[Piece], U: List[np.ndarray]):
    """Z^(1) (Eq. "stitch-temp-2") and Z^(n) (Eq. "stitch-nontemp-3") for given
    factors, without the SVD step; used to check the contractions."""
    p = len(pieces[0].V)
    rows = [pc.V[0].shape[0] for pc in pieces]
    t = np.concatenate([[0], np.cumsum(rows)]).astype(int)
    blocks = []
    for pc in pieces:
        W = pc.H
        for m in range(1, p):
            W = mode_product(W, U[m].T @ pc.V[m], m)
        blocks.append(pc.V[0] @ unfold(W, 0))
    Z = [np.vstack(blocks)]
    for n in range(1, p):
        Zn = None
        for i, pc in enumerate(pieces):
            W = mode_product(pc.H, U[0][t[i]:t[i + 1]].T @ pc.V[0], 0)
            for m in range(1, p):
                if m != n:
                    W = mode_product(W, U[m].T @ pc.V[m], m)
            W = mode_product(W, pc.V[n], n)
            term = unfold(W, n)
            Zn = term if Zn is None else Zn + term
        Z.append(Zn)
    return Z
