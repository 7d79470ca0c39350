"""Basic tensor operations, following the paper's Appendix A.

Indices start at 0.  vec() is C-order: entry (i_1..i_p) goes to position
sum_n i_n prod_{m>n} D_m.  mat_n(X) stacks the vectorised mode-n slices as
rows, so its columns run over the other indices in C-order.  The mode-n
product is defined by mat_n(G x_n U) = U mat_n(G).

Modes are 0-based in code (mode 0 is the paper's temporal mode 1).
"""

import numpy as np


def vec(X: np.ndarray) -> np.ndarray:
    """vec(X), C-order (App. A, first definition)."""
    return np.ascontiguousarray(X).reshape(-1)


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """mat_n(X): D_n x (prod of the other sizes), rows = vec of mode-n slices."""
    return np.ascontiguousarray(np.moveaxis(X, n, 0)).reshape(X.shape[n], -1)


def fold(M: np.ndarray, n: int, shape) -> np.ndarray:
    """Inverse of unfold for a tensor of the given shape."""
    shape = tuple(int(s) for s in shape)
    lead = (shape[n],) + tuple(s for i, s in enumerate(shape) if i != n)
    return np.moveaxis(M.reshape(lead), 0, n)


def mode_product(X: np.ndarray, U: np.ndarray, n: int) -> np.ndarray:
    """X x_n U, defined by mat_n(X x_n U) = U mat_n(X) (App. A)."""
    shape = list(X.shape)
    shape[n] = U.shape[0]
    return fold(U @ unfold(X, n), n, shape)


def multi_mode_product(X: np.ndarray, Us, skip=()) -> np.ndarray:
    """X x_1 U_1 x_2 U_2 ... over all modes not in ``skip`` (None entries skipped)."""
    Y = X
    for n, U in enumerate(Us):
        if n in skip or U is None:
            continue
        Y = mode_product(Y, U, n)
    return Y


def tucker_to_tensor(G: np.ndarray, Us) -> np.ndarray:
    """G x_1 U^(1) ... x_p U^(p) (the Tucker product of Eq. "tuckerals")."""
    return multi_mode_product(G, Us)


def fro2(X: np.ndarray) -> float:
    """Squared Frobenius norm (App. A, last definition)."""
    x = np.asarray(X, dtype=np.float64).reshape(-1)
    return float(x @ x)
