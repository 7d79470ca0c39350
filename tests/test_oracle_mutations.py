"""Planted mistakes in the oracle (CPU only): each must make a pin fail.

This shows the pins are sharp enough to catch a dropped term, a wrong
comparison, a transposed unfolding, the wrong end of a spectrum or a sign
error, rather than merely re-running the oracle's own formula.
"""

import numpy as np
import pytest

import oracle.stitch as S
import oracle.tucker as TK
import test_oracle_numeric as num
import test_oracle_tree as tree_pins
from oracle.tensor_ops import fold, mode_product
from oracle.tree import StreamSegmentTree


def test_trim_without_r_is_caught(monkeypatch):
    def bad_trim(H, V, a, l):
        Q, R = np.linalg.qr(V[0][a:a + l], mode="reduced")
        return S.Piece(H[:Q.shape[1]], [Q] + list(V[1:]))     # R~ dropped
    monkeypatch.setattr(S, "trim", bad_trim)
    with pytest.raises(AssertionError):
        num.test_partial_trim_represents_the_row_slice()


def test_strict_threshold_is_caught(monkeypatch):
    def strict(self, v, ts, te):
        inter = max(0, min(te, self.tau(v)) - max(ts, self.sigma(v)))
        a, b = self.theta
        return b * inter > a * (self.tau(v) - self.sigma(v))
    monkeypatch.setattr(StreamSegmentTree, "_accept", strict)
    with pytest.raises(AssertionError):
        tree_pins.test_recall_optimal_and_bounded((1, 2), 1)


def test_wrong_end_of_spectrum_is_caught(monkeypatch):
    def trailing(M, k):
        U, _, _ = np.linalg.svd(M, full_matrices=False)
        return U[:, -k:]
    monkeypatch.setattr(S, "leading_left_singular_vectors", trailing)
    with pytest.raises(AssertionError):
        num.test_stitch_full_rank_pieces_equal_hooi_on_materialised()


def test_fortran_unfolding_is_caught(monkeypatch):
    def f_unfold(X, n):
        return np.moveaxis(X, n, 0).reshape(X.shape[n], -1, order="F")
    monkeypatch.setattr(S, "unfold", f_unfold)
    with pytest.raises(AssertionError):
        num.test_contractions_match_materialised_concatenation()


def test_fit_sign_error_is_caught(monkeypatch):
    monkeypatch.setattr(S, "fit_value", lambda nx, ng: -TK.fit_value(nx, ng))
    with pytest.raises(AssertionError):
        num.test_stitch_invariants_on_noisy_pieces()


def test_dropped_sign_in_mode_product_is_caught(monkeypatch):
    orig = TK.mode_product
    monkeypatch.setattr(TK, "mode_product", lambda X, U, n: orig(X, np.abs(U), n))
    with pytest.raises(AssertionError):
        num.test_hooi_exact_recovery_and_invariants()


def test_skipped_projection_is_caught(monkeypatch):
    """HOOI that forgets to project the other modes stays at the HOSVD and
    fails the stationarity pin."""
    orig = TK.mode_product

    def lazy(X, U, n):
        # projections onto a factor (U wide) truncate instead of contracting
        if U.shape[0] < U.shape[1] and n > 0:
            idx = [slice(None)] * X.ndim
            idx[n] = slice(0, U.shape[0])
            return X[tuple(idx)]
        return orig(X, U, n)
    monkeypatch.setattr(TK, "mode_product", lazy)
    with pytest.raises(AssertionError):
        num.test_hooi_stationarity()


def test_child_order_swap_is_caught(monkeypatch):
    orig = S.stitch

    def swapped(pieces, ranks, max_iter=20, tol=0.01):
        return orig(list(reversed(pieces)), ranks, max_iter, tol)
    monkeypatch.setattr(S, "stitch", swapped)
    wl = num.synth.get("tiny")
    X = num.synth.series(wl, noise=0.0)
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=3, tol=0.0)
    for b in range(8):
        t.append(X[b * 4:(b + 1) * 4])
    with pytest.raises(AssertionError):
        for v in t.complete_nodes():
            assert num.relative_error(X[t.sigma(v):t.tau(v)], v.H, v.V) < 1e-10


def test_mode_product_reference_is_independent():
    """The elementwise pin does not go through the oracle's unfold/fold."""
    X = np.arange(24.0).reshape(2, 3, 4)
    U = np.arange(6.0).reshape(2, 3)
    Y = mode_product(X, U, 1)
    assert Y[1, 1, 2] == sum(U[1, j] * X[1, j, 2] for j in range(3))


# --- the checkers themselves (oracle/evaluate.py) -----------------------------------

import oracle.evaluate as EV  # noqa: E402
import test_oracle_evaluate as ev_pins  # noqa: E402


def test_sine_projecting_the_wrong_span_is_caught(monkeypatch):
    def own_span(A, B, k):
        Qb = np.linalg.qr(np.asarray(B, dtype=np.float64)[:, :k])[0]
        R = Qb - Qb @ (Qb.T @ Qb)                 # projects B out of its own span
        return float(np.linalg.norm(R, 2)) if R.size else 0.0
    monkeypatch.setattr(EV, "subspace_sine", own_span)
    monkeypatch.setattr(ev_pins, "subspace_sine", own_span)
    with pytest.raises(AssertionError):
        ev_pins.test_sine_of_planar_rotation(0.3)


def test_sine_smallest_angle_is_caught(monkeypatch):
    def smallest(A, B, k):
        Qa = np.linalg.qr(np.asarray(A, dtype=np.float64)[:, :k])[0]
        Qb = np.linalg.qr(np.asarray(B, dtype=np.float64)[:, :k])[0]
        s = np.linalg.svd(Qb - Qa @ (Qa.T @ Qb), compute_uv=False)
        return float(s[-1])                       # the smallest principal angle
    monkeypatch.setattr(ev_pins, "subspace_sine", smallest)
    with pytest.raises(AssertionError):
        ev_pins.test_sine_is_the_largest_angle_of_several()


def test_orthonormality_diagonal_only_is_caught(monkeypatch):
    def diag_only(U):
        U = np.asarray(U, dtype=np.float64)
        return float(np.max(np.abs(np.sum(U * U, axis=0) - 1.0)))
    monkeypatch.setattr(ev_pins, "orthonormality_error", diag_only)
    with pytest.raises(AssertionError):
        ev_pins.test_orthonormality_error_of_known_matrices()


def test_relative_error_chunk_offset_is_caught(monkeypatch):
    from oracle.tensor_ops import fro2, mode_product as mp

    def restart_rows(X, G, Us, chunk=4096):
        num_, den = 0.0, 0.0
        for t0 in range(0, X.shape[0], chunk):
            t1 = min(X.shape[0], t0 + chunk)
            Y = mp(np.asarray(G, dtype=np.float64), np.asarray(Us[0])[:t1 - t0], 0)   # rows from 0
            for n, U in enumerate(Us[1:], start=1):
                Y = mp(Y, np.asarray(U), n)
            num_ += fro2(np.asarray(X[t0:t1]) - Y)
            den += fro2(X[t0:t1])
        return float(np.sqrt(num_ / den))
    monkeypatch.setattr(ev_pins, "relative_error", restart_rows)
    with pytest.raises(AssertionError):
        ev_pins.test_relative_error_beyond_one_default_chunk()
