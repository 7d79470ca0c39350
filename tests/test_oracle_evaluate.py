"""Pins for the oracle's evaluation checkers, which gate every parity claim.

Each checker is compared with a closed form that a plausible mistake would
miss: known principal angles (a planar rotation by phi has sine sin(phi)),
a span compared with a different span of the same size (sine 1), known
non-orthonormal matrices, a reconstruction that is exact only when the
streaming chunks use the right rows of the temporal factor, errors of
exactly 1 and 1/2, and the paper's accuracy metric (Sec. 8.1) at a
scaled core, where the orthogonality of the Tucker-ALS residual to its
reconstruction fixes the value.
"""

import math

import numpy as np
import pytest
from scipy.linalg import subspace_angles

from oracle.evaluate import orthonormality_error, paper_metric, relative_error, subspace_sine
from oracle.tensor_ops import tucker_to_tensor
from oracle.tucker import hooi


def unit(n, i):
    e = np.zeros(n)
    e[i] = 1.0
    return e


# --- subspace_sine ---------------------------------------------------------------

@pytest.mark.parametrize("phi", [0.0, 1e-3, 0.3, math.pi / 4, 1.2, math.pi / 2])
def test_sine_of_planar_rotation(phi):
    A = unit(5, 0)[:, None]
    B = (math.cos(phi) * unit(5, 0) + math.sin(phi) * unit(5, 1))[:, None]
    assert abs(subspace_sine(A, B, 1) - math.sin(phi)) < 1e-13
    assert abs(subspace_sine(B, A, 1) - math.sin(phi)) < 1e-13


def test_sine_is_the_largest_angle_of_several():
    # span{e1, e2} against span{e1, cos(a) e2 + sin(a) e3}: angles 0 and a
    a = 0.7
    A = np.stack([unit(6, 0), unit(6, 1)], axis=1)
    B = np.stack([unit(6, 0), math.cos(a) * unit(6, 1) + math.sin(a) * unit(6, 2)], axis=1)
    assert abs(subspace_sine(A, B, 2) - math.sin(a)) < 1e-13
    # two rotated directions: the larger angle decides
    b = 0.2
    B2 = np.stack([math.cos(b) * unit(6, 0) + math.sin(b) * unit(6, 3),
                   math.cos(a) * unit(6, 1) + math.sin(a) * unit(6, 2)], axis=1)
    assert abs(subspace_sine(A, B2, 2) - math.sin(a)) < 1e-13


def test_sine_of_a_different_span_is_one():
    A = np.stack([unit(4, 0), unit(4, 1)], axis=1)
    B = np.stack([unit(4, 0), unit(4, 2)], axis=1)
    assert abs(subspace_sine(A, B, 2) - 1.0) < 1e-14
    # only the leading k columns count
    B3 = np.stack([unit(4, 1), unit(4, 0), unit(4, 3)], axis=1)
    assert subspace_sine(A, B3, 2) < 1e-14
    assert abs(subspace_sine(np.column_stack([A, unit(4, 2)]), B3, 3) - 1.0) < 1e-14


def test_sine_ignores_the_basis_inside_a_span():
    r = np.random.default_rng(0)
    A = np.linalg.qr(r.standard_normal((30, 5)))[0]
    M = r.standard_normal((5, 5)) + 5 * np.eye(5)  # invertible, not orthogonal
    assert subspace_sine(A, A @ M, 5) < 1e-12
    assert subspace_sine(A, -A[:, ::-1], 5) < 1e-12


def test_sine_matches_principal_angles_from_the_svd():
    r = np.random.default_rng(1)
    for _ in range(5):
        A = r.standard_normal((20, 4))
        B = A + 0.1 * r.standard_normal((20, 4))
        want = math.sin(float(np.max(subspace_angles(A, B))))
        assert abs(subspace_sine(A, B, 4) - want) < 1e-12


# --- orthonormality_error ---------------------------------------------------------

def test_orthonormality_error_of_known_matrices():
    assert orthonormality_error(np.eye(4)[:, :3]) == 0.0
    # columns of norm 1 and 2: U^T U - I = diag(0, 3)
    assert orthonormality_error(np.diag([1.0, 2.0])) == pytest.approx(3.0, abs=1e-15)
    # a shear: off-diagonal eps, diagonal eps^2
    eps = 1e-3
    U = np.array([[1.0, eps], [0.0, 1.0]])
    assert orthonormality_error(U) == pytest.approx(eps, rel=1e-12)
    # an orthonormal matrix rotated stays orthonormal
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((10, 4)))[0]
    assert orthonormality_error(Q) < 1e-14
    # a column scaled by (1 + d) is off by 2d + d^2 on the diagonal
    d = 1e-4
    Qs = Q.copy()
    Qs[:, 2] *= 1 + d
    assert orthonormality_error(Qs) == pytest.approx(2 * d + d * d, rel=1e-6)


# --- relative_error ---------------------------------------------------------------

def _exact_tucker(T, dims, ranks, seed):
    r = np.random.default_rng(seed)
    G = r.standard_normal(ranks)
    Us = [r.standard_normal((T, ranks[0]))] + [np.linalg.qr(r.standard_normal((D, k)))[0]
                                              for D, k in zip(dims, ranks[1:])]
    return G, Us, tucker_to_tensor(G, Us)


@pytest.mark.parametrize("chunk", [1, 7, 16, 4096])
def test_relative_error_exact_across_chunks(chunk):
    # an exact decomposition: every chunk must use its own rows of U^(1)
    T = 2 * 16 + 5
    G, Us, X = _exact_tucker(T, (4, 3), (3, 2, 2), 3)
    assert relative_error(X, G, Us, chunk=chunk) < 1e-14
    # rows of U^(1) shifted by one: the same mistake a chunk offset would make
    Ush = [np.roll(Us[0], 1, axis=0)] + Us[1:]
    assert relative_error(X, G, Ush, chunk=chunk) > 0.1


def test_relative_error_beyond_one_default_chunk():
    # more than 4096 slices with the default chunk: exact decomposition -> 0,
    # plus a perturbation confined to the second chunk with a known norm
    T = 4096 + 300
    G, Us, X = _exact_tucker(T, (3, 2), (2, 2, 2), 4)
    assert relative_error(X, G, Us) < 1e-14
    E = np.zeros_like(X)
    E[4100:4200] = np.random.default_rng(5).standard_normal((100, 3, 2))
    Xp = X + E
    want = math.sqrt(float(np.sum(E * E)) / float(np.sum(Xp * Xp)))
    assert relative_error(Xp, G, Us) == pytest.approx(want, rel=1e-12)


def test_relative_error_closed_forms():
    G, Us, X = _exact_tucker(50, (5, 4), (3, 3, 2), 6)
    assert relative_error(X, 0.0 * G, Us) == pytest.approx(1.0, abs=1e-15)
    assert relative_error(X, 0.5 * G, Us, chunk=9) == pytest.approx(0.5, rel=1e-13)
    assert relative_error(X, 3.0 * G, Us, chunk=11) == pytest.approx(2.0, rel=1e-13)


# --- paper_metric (Sec. 8.1: |X - Y_A| / |X - Y_ALS| - 1) ---------------------------

def test_paper_metric_closed_forms():
    r = np.random.default_rng(7)
    _, _, Y = _exact_tucker(12, (6, 5), (3, 3, 2), 8)
    X = Y + 0.05 * r.standard_normal(Y.shape)
    ranks = (3, 3, 2)
    G, Us, _ = hooi(X, ranks, 20, 0.0)
    # the from-scratch decomposition itself scores 0
    assert abs(paper_metric(X, G, Us, ranks, 20, 0.0)) < 1e-12
    # a scaled core: the ALS residual is orthogonal to its reconstruction, so
    # |X - c Y^|^2 = |X - Y^|^2 + (1 - c)^2 |Y^|^2
    Yh = tucker_to_tensor(G, Us)
    e2 = float(np.sum((X - Yh) ** 2))
    c = 0.9
    want = math.sqrt(e2 + (1 - c) ** 2 * float(np.sum(Yh * Yh))) / math.sqrt(e2) - 1.0
    assert paper_metric(X, c * G, Us, ranks, 20, 0.0) == pytest.approx(want, rel=1e-9)
    # a zero decomposition: |X| / |X - Y_ALS| - 1
    want0 = math.sqrt(float(np.sum(X * X)) / e2) - 1.0
    assert paper_metric(X, 0 * G, Us, ranks, 20, 0.0) == pytest.approx(want0, rel=1e-9)
