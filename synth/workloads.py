"""Synthetic tensor time series shaped like the paper's workloads.

The paper evaluates on real datasets (time x location x pollutant, time x
frequency x sensor, time x company x feature; Sec. 8, Table "Description")
that are not available here.  These generators stand in for them: a low
Tucker-rank signal plus noise, with a tall temporal mode, one large "entity"
mode and one small "feature" mode.

Recipe (all FP64, NumPy PCG64):
  * non-temporal factors B^(n) (D_n x q_n): orthonormalised Gaussians, or
    |N(0,1)| entries (not orthonormalised) for the non-negative workload;
  * core G (q_1 x ... x q_p): N(0,1), or exp(N(0,1)) for the non-negative one;
  * temporal factor row t: xi_t * m_{floor(t/P)} with xi_t ~ N(0, I) (|.| for
    the non-negative one) and m_k a 0/1 mask with ceil(q_1/2) ones per regime,
    so that a short range has lower temporal rank and different loadings;
  * W = G x_1 A x_2 B^(2) ... scaled to unit RMS (scale measured on the first
    min(T, 1024) slices so that any prefix can be generated on its own);
  * additive noise X = W + sigma N(0,1), or multiplicative
    X = W * exp(sigma xi - sigma^2/2) for the non-negative workload;
  * drifting workload: B^(n)(t) = orth(cos(w t) B0 + sin(w t) B1) with
    w = (pi/2)/T_max, i.e. a quarter turn over the whole stream.

Random draws for slices are made per chunk of CHUNK slices from
SeedSequence([seed, chunk]), so any time range can be produced without
generating what precedes it; the noise of large slices is drawn in chunks
of fewer slices (at most NOISE_CHUNK_ELEMS elements a chunk).  FP32 workloads are rounded to FP32 and promoted
back to FP64, so the oracle sees exactly the values the GPU sees.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

CHUNK = 256
NOISE_CHUNK_ELEMS = 1 << 24


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: Tuple[int, ...]            # non-temporal sizes D_2..D_p
    T: int                           # timespan
    true_ranks: Tuple[int, ...]      # q_1..q_p of the generator
    noise: float
    leaf_len: int
    node_ranks: Tuple[int, ...]      # r_1..r_p
    n_queries: int
    query_kind: str                  # "pairs" | "uniform_len" | "loguniform"
    min_len: int = 1
    regime: Optional[int] = None     # regime period P (None: a single regime)
    nonneg: bool = False
    drift: bool = False
    dtype: str = "f32"               # "f64" | "f32"
    theta: Tuple[int, int] = (7, 10)
    max_iter: int = 20
    tol: float = 0.01
    seed: int = 0

    @property
    def p(self) -> int:
        return 1 + len(self.dims)

    @property
    def query_seed(self) -> int:
        return self.seed + 1000


WORKLOADS = {
    # 3-way FP64 20x20xT=256, true rank (4,4,4), regimes every 64 steps.
    "tiny": Workload("tiny", (20, 20), 256, (4, 4, 4), 0.01, 4, (5, 5, 5), 32,
                     "pairs", regime=64, dtype="f64", seed=1001),
    # 64x64xT=4096 FP32, true rank (8,8,8), 8 regimes; one query per launch.
    "plain": Workload("plain", (64, 64), 4096, (8, 8, 8), 0.05, 8, (10, 10, 10),
                      2048, "uniform_len", regime=512, seed=1002),
    # 128x96xT=16384 FP32, true rank 12; 4096 log-uniform queries in [16, T].
    "batch": Workload("batch", (128, 96), 16384, (12, 12, 12), 0.05, 16,
                      (16, 16, 16), 4096, "loguniform", min_len=16, seed=1003),
    # 4-way day x location x hour x feature, non-negative log-normal.
    "precision": Workload("precision", (200, 24, 8), 32768, (20, 20, 6, 4), 0.1,
                          1, (20, 20, 6, 4), 1024, "loguniform", regime=365,
                          nonneg=True, seed=1004),
    # 128x128 slices, drifting rank-16 model, T grows to 65536.
    "serving": Workload("serving", (128, 128), 65536, (16, 16, 16), 0.05, 1,
                        (16, 16, 16), 4096, "loguniform", drift=True, seed=1005),
}


# The paper's many-mode shapes (every slice 10^6 elements; time first):
# 1000x1000, 100x100x100, 100x100x10x10, 100x10x10x10x10 (and a sixth
# non-temporal mode of 10 at p = 7), rank 5 in every mode, here over 400
# slices of one regime so that queries of 98, 192 and 384 slices fit.
D5_SHAPES = {3: (1000, 1000), 4: (100, 100, 100), 5: (100, 100, 10, 10), 6: (100, 10, 10, 10, 10),
             7: (10, 10, 10, 10, 10, 10)}


def d5(p: int, T: int = 400) -> Workload:
    dims = D5_SHAPES[p]
    name = "d5_p%d" % p if T == 400 else "d5_p%d_T%d" % (p, T)
    return Workload(name, dims, T, (5,) * p, 0.05, 1, (5,) * p, 256, "uniform_len", seed=3000 + p)


def get(name: str) -> Workload:
    """A workload by name: the table above, or d5_p<p> / d5_p<p>_T<T>."""
    if name.startswith("d5_p"):
        parts = name[4:].split("_T")
        return d5(int(parts[0]), int(parts[1]) if len(parts) > 1 else 400)
    return WORKLOADS[name]


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *key])))


def _static(wl: Workload):
    """Factors, core, drift partners and regime masks (all time-independent)."""
    rng = _rng(wl.seed, 0)
    q = wl.true_ranks
    B0, B1 = [], []
    for D, qn in zip(wl.dims, q[1:]):
        if wl.nonneg:
            B0.append(np.abs(rng.standard_normal((D, qn))))
            B1.append(None)
        else:
            B0.append(np.linalg.qr(rng.standard_normal((D, qn)))[0])
            B1.append(np.linalg.qr(rng.standard_normal((D, qn)))[0] if wl.drift else None)
    G = rng.standard_normal(q)
    if wl.nonneg:
        G = np.exp(G)
    n_reg = 1 if wl.regime is None else -(-wl.T // wl.regime)
    masks = np.ones((n_reg, q[0]))
    if wl.regime is not None:
        ones = -(-q[0] // 2)
        for k in range(n_reg):
            m = np.zeros(q[0])
            m[rng.choice(q[0], size=ones, replace=False)] = 1.0
            masks[k] = m
    return B0, B1, G, masks


def _signal(wl: Workload, st, t0: int, t1: int) -> np.ndarray:
    B0, B1, G, masks = st
    rng = None
    out = np.empty((t1 - t0,) + wl.dims)
    c0 = t0 // CHUNK
    for c in range(c0, -(-t1 // CHUNK)):
        lo, hi = max(t0, c * CHUNK), min(t1, (c + 1) * CHUNK)
        rng = _rng(wl.seed, 1, c)
        xi = rng.standard_normal((CHUNK, wl.true_ranks[0]))[lo - c * CHUNK:hi - c * CHUNK]
        if wl.nonneg:
            xi = np.abs(xi)
        t = np.arange(lo, hi)
        reg = np.zeros_like(t) if wl.regime is None else t // wl.regime
        A = xi * masks[reg]
        if wl.drift:
            for i, tt in enumerate(t):
                w = (math.pi / 2.0) * tt / wl.T
                Bs = [np.linalg.qr(math.cos(w) * b0 + math.sin(w) * b1)[0]
                      for b0, b1 in zip(B0, B1)]
                out[lo - t0 + i] = _expand(G, A[i:i + 1], Bs)[0]
        else:
            out[lo - t0:hi - t0] = _expand(G, A, B0)
    return out


def _expand(G, A, Bs) -> np.ndarray:
    """Y = G x_1 A x_2 B^(2) ... written with plain einsum-free reshapes."""
    Y = np.tensordot(A, G, axes=([1], [0]))           # (t, q2, ..., qp)
    for n, B in enumerate(Bs, start=1):
        Y = np.moveaxis(np.tensordot(Y, B, axes=([n], [1])), -1, n)
    return Y


def _noise_chunk(wl: Workload) -> int:
    return max(1, min(CHUNK, NOISE_CHUNK_ELEMS // math.prod(wl.dims)))


def _noise(wl: Workload, t0: int, t1: int) -> np.ndarray:
    out = np.empty((t1 - t0,) + wl.dims)
    ch = _noise_chunk(wl)
    for c in range(t0 // ch, -(-t1 // ch)):
        lo, hi = max(t0, c * ch), min(t1, (c + 1) * ch)
        rng = _rng(wl.seed, 2, c)
        e = rng.standard_normal((ch,) + wl.dims)
        out[lo - t0:hi - t0] = e[lo - c * ch:hi - c * ch]
    return out


_SCALE_CACHE = {}


def _scale(wl: Workload, st) -> float:
    key = (wl.name, wl.seed, wl.T, wl.dims, wl.true_ranks)
    if key not in _SCALE_CACHE:
        n = min(wl.T, 1024)
        W = _signal(wl, st, 0, n)
        rms = math.sqrt(float(np.mean(W * W)))
        _SCALE_CACHE[key] = 1.0 / rms if rms > 0 else 1.0
    return _SCALE_CACHE[key]


def series(wl: Workload, t0: int = 0, t1: Optional[int] = None,
           noise: Optional[float] = None) -> np.ndarray:
    """Slices [t0, t1) of the workload's tensor series, FP64 (FP32-exact for
    FP32 workloads).  ``noise`` overrides the workload's noise level."""
    t1 = wl.T if t1 is None else t1
    assert 0 <= t0 <= t1
    st = _static(wl)
    W = _signal(wl, st, t0, t1) * _scale(wl, st)
    sigma = wl.noise if noise is None else noise
    if sigma > 0:
        E = _noise(wl, t0, t1)
        if wl.nonneg:
            X = W * np.exp(sigma * E - 0.5 * sigma * sigma)
        else:
            X = W + sigma * E
    else:
        X = W
    if wl.dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
    return X


def queries(wl: Workload, T: Optional[int] = None, n: Optional[int] = None,
            seed_offset: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded query ranges [ts, te) over [0, T) following the workload's
    length distribution."""
    T = wl.T if T is None else T
    n = wl.n_queries if n is None else n
    rng = _rng(wl.query_seed + seed_offset, 0)
    ts = np.empty(n, dtype=np.int64)
    te = np.empty(n, dtype=np.int64)
    for i in range(n):
        if wl.query_kind == "pairs":
            a, b = sorted(rng.choice(T + 1, size=2, replace=False))
            ts[i], te[i] = a, b
            continue
        if wl.query_kind == "uniform_len":
            L = int(rng.integers(1, T + 1))
        else:
            lo = max(1, min(wl.min_len, T))
            L = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(T)))))
            L = min(max(L, lo), T)
        s = int(rng.integers(0, T - L + 1))
        ts[i], te[i] = s, s + L
    return ts, te


def small_series(shape: Sequence[int], ranks: Sequence[int], noise: float,
                 seed: int, orthonormal: bool = True) -> np.ndarray:
    """A small low-rank-plus-noise tensor of any order for unit tests."""
    rng = _rng(seed, 7)
    G = rng.standard_normal(tuple(ranks))
    Y = G
    for n, (D, r) in enumerate(zip(shape, ranks)):
        B = rng.standard_normal((D, r))
        if orthonormal:
            B = np.linalg.qr(B)[0]
        Y = np.moveaxis(np.tensordot(Y, B, axes=([n], [1])), -1, n)
    Y = Y / math.sqrt(float(np.mean(Y * Y)))
    return Y + noise * rng.standard_normal(tuple(shape))
