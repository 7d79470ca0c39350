"""Pins for the oracle's tensor algebra, Tucker-ALS, trims and Stitch.

Each check compares against something other than the oracle's own formula:
index-by-index definitions (App. A), LAPACK's SVD of a matrix (Eckart-Young),
materialised tensors, exact recovery of noise-free low-rank data, the norm
identity of an orthogonal projection, monotone ALS fits, and the error bound
of Prop. "err".
"""

import itertools
import math

import numpy as np
import pytest

import synth
from oracle import stitch as S
from oracle.evaluate import orthonormality_error, relative_error, subspace_sine
from oracle.tensor_ops import fold, fro2, mode_product, tucker_to_tensor, unfold, vec
from oracle.tree import StreamSegmentTree
from oracle.tucker import canonical_signs, effective_ranks, hooi


def rng(seed):
    return np.random.default_rng(seed)


# --- App. A definitions, index by index ----------------------------------------

def test_vec_c_order():
    X = rng(0).standard_normal((2, 3, 4))
    v = vec(X)
    for i, j, k in itertools.product(range(2), range(3), range(4)):
        assert v[i * 12 + j * 4 + k] == X[i, j, k]


def test_unfold_rows_are_vectorised_slices():
    X = rng(1).standard_normal((2, 3, 4, 5))
    for n in range(4):
        M = unfold(X, n)
        for i in range(X.shape[n]):
            sl = [slice(None)] * 4
            sl[n] = i
            assert np.array_equal(M[i], X[tuple(sl)].reshape(-1))
        assert np.array_equal(fold(M, n, X.shape), X)


def test_mode_product_elementwise():
    X = rng(2).standard_normal((2, 3, 4))
    U = rng(3).standard_normal((5, 3))
    Y = mode_product(X, U, 1)
    assert Y.shape == (2, 5, 4)
    for a, i, b in itertools.product(range(2), range(5), range(4)):
        assert abs(Y[a, i, b] - sum(U[i, j] * X[a, j, b] for j in range(3))) < 1e-12
    # reverse associativity (Sec. 5.1 footnote): X x_n A x_n B = X x_n (B A)
    A = rng(4).standard_normal((6, 3))
    B = rng(5).standard_normal((2, 6))
    assert np.allclose(mode_product(mode_product(X, A, 1), B, 1), mode_product(X, B @ A, 1))
    assert abs(fro2(X) - sum(x * x for x in X.reshape(-1))) < 1e-12


# --- effective ranks -------------------------------------------------------------

def test_effective_ranks():
    assert effective_ranks(1, (128, 128), (16, 16, 16)) == (1, 16, 16)
    assert effective_ranks(1, (200, 24, 8), (20, 20, 6, 4)) == (1, 20, 6, 4)
    assert effective_ranks(4, (20, 20), (5, 5, 5)) == (4, 5, 5)
    assert effective_ranks(1, (20, 3), (5, 5, 5)) == (1, 3, 3)
    assert effective_ranks(2, (1, 9), (5, 5, 5)) == (2, 1, 2)
    assert effective_ranks(3, (2, 2), (5, 5, 5)) == (3, 2, 2)
    assert effective_ranks(1, (1, 9), (5, 5, 5)) == (1, 1, 1)
    assert effective_ranks(16384, (128, 96), (16, 16, 16)) == (16, 16, 16)


# --- Tucker-ALS --------------------------------------------------------------------

def test_hooi_on_matrix_is_truncated_svd():
    M = rng(6).standard_normal((30, 12))
    G, U, _ = hooi(M, (4, 4), max_iter=5, tol=0.0)
    s = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(np.sort(np.abs(np.linalg.svd(G, compute_uv=False)))[::-1], s[:4])
    err2 = fro2(M - tucker_to_tensor(G, U))
    assert abs(err2 - np.sum(s[4:] ** 2)) < 1e-10 * fro2(M)


def test_leaf_single_slice_is_truncated_svd():
    """l = 1, p = 3: the leaf decomposition is the truncated SVD of the slice."""
    X = rng(7).standard_normal((1, 15, 11))
    r = effective_ranks(1, (15, 11), (5, 5, 5))
    G, U, _ = hooi(X, r, max_iter=3, tol=0.0)
    G, U = canonical_signs(G, U)
    Uu, s, Vt = np.linalg.svd(X[0])
    assert np.allclose(np.abs(G[0]), np.diag(s[:r[1]]), atol=1e-10)
    assert subspace_sine(U[1], Uu, r[1]) < 1e-10
    assert subspace_sine(U[2], Vt.T, r[2]) < 1e-10


def test_hooi_exact_recovery_and_invariants():
    X = synth.small_series((9, 8, 7), (3, 2, 3), 0.0, seed=1)
    G, U, info = hooi(X, (3, 2, 3), max_iter=4, tol=0.0)
    assert relative_error(X, G, U) < 1e-12
    for Un in U:
        assert orthonormality_error(Un) < 1e-12
    Xn = synth.small_series((9, 8, 7), (3, 2, 3), 0.1, seed=2)
    G, U, info = hooi(Xn, (3, 2, 3), max_iter=6, tol=0.0)
    # norm identity: |X|^2 - |G|^2 = |X - Y^|^2 (orthogonal projection)
    assert abs(fro2(Xn) - fro2(G) - fro2(Xn - tucker_to_tensor(G, U))) < 1e-10 * fro2(Xn)
    # monotone fit
    assert all(b >= a - 1e-12 for a, b in zip(info["fits"], info["fits"][1:]))


def test_hooi_stationarity():
    """At convergence each U^(n) spans the leading left singular subspace of
    mat_n(X x_{m != n} U^(m)T) (Eq. "als-mat"), checked with an independent
    SVD, and the ALS error is below the HOSVD error."""
    X = synth.small_series((10, 9, 8), (3, 3, 3), 0.3, seed=4)
    r = (3, 3, 3)
    G, U, info = hooi(X, r, max_iter=60, tol=0.0)
    for n in range(3):
        # contract the two other modes slice by slice, without unfold/fold
        M = np.zeros((X.shape[n], r[(n + 1) % 3] * r[(n + 2) % 3]))
        a, b = sorted([(n + 1) % 3, (n + 2) % 3])
        for i in range(X.shape[n]):
            sl = [slice(None)] * 3
            sl[n] = i
            M[i] = (U[a].T @ X[tuple(sl)] @ U[b]).reshape(-1)
        Ul = np.linalg.svd(M, full_matrices=False)[0][:, :r[n]]
        assert subspace_sine(U[n], Ul, r[n]) < 1e-6
    Uh = [np.linalg.svd(unfold(X, n), full_matrices=False)[0][:, :r[n]] for n in range(3)]
    Gh = X
    for n in range(3):
        Gh = mode_product(Gh, Uh[n].T, n)
    assert relative_error(X, G, U) <= relative_error(X, Gh, Uh) + 1e-12


# --- trims and stitching on explicit pieces ---------------------------------------------

def _random_piece(r, rows, k, dims, ranks):
    V1 = np.linalg.qr(r.standard_normal((rows, k)))[0]
    Vs = [np.linalg.qr(r.standard_normal((D, q)))[0] for D, q in zip(dims, ranks)]
    H = r.standard_normal((k,) + tuple(ranks))
    return S.Piece(H, [V1] + Vs)


def _materialise(pieces):
    return np.concatenate([tucker_to_tensor(pc.H, pc.V) for pc in pieces], axis=0)


def test_partial_trim_represents_the_row_slice():
    r = rng(8)
    pc = _random_piece(r, 12, 4, (6, 5), (3, 2))
    Y = tucker_to_tensor(pc.H, pc.V)
    for a, l in [(0, 9), (3, 9), (2, 3), (11, 1)]:
        tp = S.trim(pc.H, pc.V, a, l)
        Q = tp.V[0]
        assert orthonormality_error(Q) < 1e-13
        assert np.allclose(tucker_to_tensor(tp.H, tp.V), Y[a:a + l], atol=1e-13)


def test_contractions_match_materialised_concatenation():
    """Eqs. "stitch-temp-2" and "stitch-nontemp-3" equal
    mat_n(Y~) (kron_{m != n} U^(m)) computed on the materialised Y~."""
    r = rng(9)
    dims, ranks = (7, 6, 5), (3, 2, 4)
    pieces = [_random_piece(r, rows, k, dims, ranks) for rows, k in [(5, 3), (8, 4), (2, 2)]]
    Y = _materialise(pieces)
    out = (3, 2, 2, 3)
    U = [np.linalg.qr(r.standard_normal((Y.shape[n], out[n])))[0] for n in range(4)]
    Z = S.z_matrices(pieces, U)
    for n in range(4):
        W = Y
        for m in range(4):
            if m != n:
                W = mode_product(W, U[m].T, m)
        assert np.allclose(Z[n], unfold(W, n), atol=1e-12)
        if n > 0:
            Gm = unfold(Y, n) @ unfold(Y, n).T
            assert np.allclose(S._gram_hosvd(pieces, n), Gm, atol=1e-11)
    assert abs(S.ytilde_norm2(pieces) - fro2(Y)) < 1e-11 * fro2(Y)


def test_stitch_full_rank_pieces_equal_hooi_on_materialised():
    """Pieces that represent X exactly: Stitch == Tucker-ALS on X, sweep for sweep."""
    X = synth.small_series((14, 6, 5), (4, 3, 3), 0.2, seed=3)
    cuts = [0, 4, 9, 14]
    pieces = []
    for a, b in zip(cuts, cuts[1:]):
        Gp, Up, _ = hooi(X[a:b], (b - a, 6, 5), max_iter=1, tol=0.0)
        pieces.append(S.Piece(Gp, Up))
    assert np.allclose(_materialise(pieces), X, atol=1e-12)
    for sweeps in (1, 3):
        G1, U1, _ = S.stitch(pieces, (3, 3, 2), max_iter=sweeps, tol=0.0)
        G2, U2, _ = hooi(X, (3, 3, 2), max_iter=sweeps, tol=0.0)
        G2, U2 = canonical_signs(G2, U2)
        assert np.allclose(tucker_to_tensor(G1, U1), tucker_to_tensor(G2, U2), atol=1e-10)
        for a, b in zip(U1, U2):
            assert subspace_sine(a, b, a.shape[1]) < 1e-9
        assert np.allclose(G1, G2, atol=1e-9)


@pytest.mark.parametrize("shape,ranks", [
    ((6, 4, 3, 3, 2), (2, 2, 2, 2, 2)),
    ((6, 3, 3, 2, 2, 2, 2), (2, 2, 2, 2, 2, 2, 2)),
])
def test_many_modes_exact_recovery_and_stitch(shape, ranks):
    """Five and seven modes: exact Tucker data is recovered to rounding, and
    the stitch of pieces that represent X exactly equals Tucker-ALS on X."""
    X = synth.small_series(shape, ranks, 0.0, seed=11)
    G, U, _ = hooi(X, ranks, max_iter=3, tol=0.0)
    assert relative_error(X, G, U) < 1e-11
    Xn = synth.small_series(shape, ranks, 0.2, seed=12)
    pieces = []
    for a, b in ((0, 2), (2, 6)):
        Gp, Up, _ = hooi(Xn[a:b], (b - a,) + shape[1:], max_iter=1, tol=0.0)
        pieces.append(S.Piece(Gp, Up))
    assert np.allclose(_materialise(pieces), Xn, atol=1e-12)
    G1, U1, _ = S.stitch(pieces, ranks, max_iter=2, tol=0.0)
    G2, U2, _ = hooi(Xn, ranks, max_iter=2, tol=0.0)
    assert np.allclose(tucker_to_tensor(G1, U1), tucker_to_tensor(G2, U2), atol=1e-10)
    for a, b in zip(U1, U2):
        assert subspace_sine(a, b, a.shape[1]) < 1e-9


def test_stitch_invariants_on_noisy_pieces():
    r = rng(10)
    dims, ranks = (9, 7), (4, 3)
    pieces = [_random_piece(r, rows, k, dims, ranks) for rows, k in [(6, 4), (10, 4), (3, 3)]]
    Y = _materialise(pieces)
    G, U, info = S.stitch(pieces, (4, 4, 3), max_iter=8, tol=0.0)
    for Un in U:
        assert orthonormality_error(Un) < 1e-12
    # core = Y~ x_n U^(n)T, and the norm identity
    Gd = Y
    for n in range(3):
        Gd = mode_product(Gd, U[n].T, n)
    assert np.allclose(G, Gd, atol=1e-12)
    assert abs(info["err_model"] ** 2 * fro2(Y) - fro2(Y - tucker_to_tensor(G, U))) < 1e-10 * fro2(Y)
    assert all(b >= a - 1e-12 for a, b in zip(info["fits"], info["fits"][1:]))


# --- end to end on the tiny workload -----------------------------------------------------

@pytest.fixture(scope="module")
def tiny_tree_noise_free():
    wl = synth.get("tiny")
    X = synth.series(wl, noise=0.0)
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=6, tol=0.0)
    for b in range(wl.T // wl.leaf_len):
        t.append(X[b * wl.leaf_len:(b + 1) * wl.leaf_len])
    return wl, X, t


def test_exact_recovery_every_node_and_query(tiny_tree_noise_free):
    wl, X, t = tiny_tree_noise_free
    for v in t.complete_nodes():
        Xi = X[t.sigma(v):t.tau(v)]
        assert relative_error(Xi, v.H, v.V) < 1e-10
    ts, te = synth.queries(wl)
    for a, b in zip(ts, te):
        G, U, info = t.query(int(a), int(b))
        assert relative_error(X[a:b], G, U) < 1e-10
        for Un in U:
            assert orthonormality_error(Un) < 1e-12


def test_single_node_range_returns_the_node(tiny_tree_noise_free):
    wl, X, t = tiny_tree_noise_free
    for v in t.complete_nodes()[::3]:
        G, U, info = t.query(t.sigma(v), t.tau(v))
        assert info["sweeps"] == 0
        assert np.array_equal(G, v.H) and all(np.array_equal(a, b) for a, b in zip(U, v.V))


def test_query_output_ranks(tiny_tree_noise_free):
    """Output ranks below the nodes' (Alg. "stitch" takes the target ranks
    as an input).  Noise-free tiny data has multilinear rank (4, 4, 4) and the
    nodes hold (5, 5, 5): asking for (4, 4, 4) still reconstructs every query
    exactly, (3, 3, 3) leaves a positive error with factors of 3 columns, and
    a stored node's own range at reduced ranks goes through the stitch and
    agrees with Tucker-ALS on the node's materialised tensor."""
    wl, X, t = tiny_tree_noise_free
    ts, te = synth.queries(wl)
    for a, b in list(zip(ts.tolist(), te.tolist()))[:12]:
        G4, U4, _ = t.query(a, b, ranks=wl.true_ranks)
        assert G4.shape == effective_ranks(b - a, wl.dims, wl.true_ranks)
        assert relative_error(X[a:b], G4, U4) < 1e-10
        G3, U3, _ = t.query(a, b, ranks=(3, 3, 3))
        assert all(Un.shape[1] == min(3, Un.shape[0]) for Un in U3)
        if b - a >= 4:
            assert relative_error(X[a:b], G3, U3) > 1e-6
        for Un in U3:
            assert orthonormality_error(Un) < 1e-12
    for v in t.complete_nodes():
        if (t.tau(v) - t.sigma(v)) >= 16:
            break
    G, U, info = t.query(t.sigma(v), t.tau(v), max_iter=3, tol=0.0, ranks=(3, 3, 3))
    assert info["sweeps"] == 3
    Gh, Uh, _ = hooi(tucker_to_tensor(v.H, v.V), (3, 3, 3), max_iter=3, tol=0.0)
    assert np.allclose(tucker_to_tensor(G, U), tucker_to_tensor(Gh, Uh), atol=1e-9)
    with pytest.raises(ValueError):
        t.query(0, 8, ranks=(6, 5, 5))


def test_fixed_block_queries_recover_noise_free_data(tiny_tree_noise_free):
    """Queries stitched from the fixed-block hit set (level 2: blocks of 16
    slices) reconstruct noise-free data exactly, like Alg. "recall"'s."""
    wl, X, t = tiny_tree_noise_free
    ts, te = synth.queries(wl)
    for a, b in list(zip(ts.tolist(), te.tolist()))[:16]:
        G, U, info = t.query(a, b, level=2)
        assert all(t.tau(v) - t.sigma(v) == 4 * wl.leaf_len for v, lo, hi in info["hits"][:-1])
        assert relative_error(X[a:b], G, U) < 1e-10


def test_tail_queries_recover_noise_free_data():
    """Ranges reaching into an incomplete block take that block's provisional
    piece (the leaf procedure on its slices), trimmed like a partial hit.
    Noise-free tiny data, 63 complete blocks of 4 slices and a tail of 3:
    every range ending in the tail reconstructs exactly, ranges inside the
    tail included; a range inside the committed part is unaffected."""
    wl = synth.get("tiny")
    X = synth.series(wl, noise=0.0)
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, max_iter=6, tol=0.0)
    for b in range(63):
        t.append(X[b * wl.leaf_len:(b + 1) * wl.leaf_len])
    Tc = t.T
    tail = X[Tc:Tc + 3]
    for a, c in [(0, 255), (100, 253), (250, 254), (252, 255), (253, 255), (254, 255)]:
        G, U, info = t.query(a, c, tail=tail)
        assert info["tail"] == (max(a, Tc), c)
        assert relative_error(X[a:c], G, U) < 1e-10
        for Un in U:
            assert orthonormality_error(Un) < 1e-12
    G1, U1, _ = t.query(10, 200)
    G2, U2, _ = t.query(10, 200, tail=tail)
    assert np.array_equal(G1, G2) and all(np.array_equal(a, b) for a, b in zip(U1, U2))
    with pytest.raises(ValueError):
        t.query(0, Tc + 4, tail=tail)


def test_error_bound_on_noisy_tiny():
    """Prop. "err": |X - Y| / |X| <= 3 eps when X = W + E, eps = |E|/|X|."""
    wl = synth.get("tiny")
    X = synth.series(wl)
    W = synth.series(wl, noise=0.0)
    t = StreamSegmentTree(wl.dims, wl.node_ranks, wl.leaf_len, wl.theta, wl.max_iter, wl.tol)
    for b in range(wl.T // wl.leaf_len):
        t.append(X[b * wl.leaf_len:(b + 1) * wl.leaf_len])
    ts, te = synth.queries(wl)
    for a, b in zip(ts, te):
        G, U, info = t.query(int(a), int(b))
        eps = math.sqrt(fro2(X[a:b] - W[a:b]) / fro2(X[a:b]))
        assert relative_error(X[a:b], G, U) <= 3 * eps
        for Un in U:
            assert orthonormality_error(Un) < 1e-12


# --- the exact reductions the GPU path relies on -------------------------------------------

def test_temporal_reduction_identity():
    """Left singular vectors of Z^(1) = blockdiag(V~_i^(1)) x those of the
    stacked small matrix M = [mat_1(W_i)]_i (the V~_i^(1) are orthonormal)."""
    r = rng(11)
    dims, ranks = (8, 6), (3, 3)
    pieces = [_random_piece(r, rows, k, dims, ranks) for rows, k in [(7, 3), (12, 3), (4, 2)]]
    U = [None] + [np.linalg.qr(r.standard_normal((D, 3)))[0] for D in dims]
    U[0] = np.zeros((23, 3))
    Z1 = S.z_matrices(pieces, U)[0]
    Ms = []
    for pc in pieces:
        W = pc.H
        for m in (1, 2):
            W = mode_product(W, U[m].T @ pc.V[m], m)
        Ms.append(unfold(W, 0))
    M = np.vstack(Ms)
    P = np.linalg.svd(M, full_matrices=False)[0][:, :3]
    rows = np.cumsum([0] + [pc.V[0].shape[0] for pc in pieces])
    ks = np.cumsum([0] + [pc.V[0].shape[1] for pc in pieces])
    U1 = np.vstack([pc.V[0] @ P[ks[i]:ks[i + 1]] for i, pc in enumerate(pieces)])
    assert rows[-1] == U1.shape[0]
    assert subspace_sine(np.linalg.svd(Z1, full_matrices=False)[0], U1, 3) < 1e-10


def test_nontemporal_basis_reduction_identity():
    """With B an orthonormal basis of span[V~_1^(n), ..., V~_s^(n)],
    Z^(n) = B (B^T Z^(n)), so its leading left singular vectors are B times
    those of the small matrix B^T Z^(n)."""
    r = rng(12)
    dims, ranks = (40, 6), (3, 3)
    pieces = [_random_piece(r, rows, 3, dims, ranks) for rows in (7, 9)]
    U = [np.linalg.qr(r.standard_normal((16, 3)))[0]] + \
        [np.linalg.qr(r.standard_normal((D, 3)))[0] for D in dims]
    Z = S.z_matrices(pieces, U)[1]
    Vcat = np.hstack([pc.V[1] for pc in pieces])
    w, E = np.linalg.eigh(Vcat.T @ Vcat)
    keep = w > 1e-10 * w.max()
    B = Vcat @ E[:, keep] / np.sqrt(w[keep])
    assert orthonormality_error(B) < 1e-12
    Pk = np.linalg.svd(B.T @ Z, full_matrices=False)[0][:, :3]
    assert subspace_sine(np.linalg.svd(Z, full_matrices=False)[0], B @ Pk, 3) < 1e-10
