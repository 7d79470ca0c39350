"""Python binding of libtucket (include/tucket.h): argument marshalling only.

Every step of build, append and query runs in the HIP library; this module
allocates device buffers through PyTorch, passes pointers and sizes, and
turns status codes into exceptions.  It fails loudly when the library has
not been built (there is no fallback).
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtucket.so")
MAX_MODES = 8

TK_OK, TK_EINVAL, TK_ERANGE, TK_ENOMEM, TK_EDEVICE, TK_EBUSY = range(6)
TK_F32, TK_BF16 = 1, 2
_STATUS = {TK_EINVAL: "TK_EINVAL", TK_ERANGE: "TK_ERANGE", TK_ENOMEM: "TK_ENOMEM",
           TK_EDEVICE: "TK_EDEVICE", TK_EBUSY: "TK_EBUSY"}

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class TkConfig(ctypes.Structure):
    _fields_ = [("p", c_i32), ("dims", c_i64 * MAX_MODES), ("ranks", c_i32 * MAX_MODES),
                ("leaf_len", c_i32), ("theta_num", c_i32), ("theta_den", c_i32),
                ("max_iter", c_i32), ("tol", c_dbl), ("prec", c_i32),
                ("capacity_T", c_i64), ("mem_budget_bytes", c_i64)]


class TkHit(ctypes.Structure):
    _fields_ = [("level", c_i32), ("partial", c_i32), ("index", c_i64), ("node_id", c_i64),
                ("sigma", c_i64), ("tau", c_i64), ("lo", c_i64), ("hi", c_i64)]


class TkShape(ctypes.Structure):
    _fields_ = [("ranks_eff", c_i32 * MAX_MODES), ("L", c_i64), ("core_elems", c_i64),
                ("factor_elems", c_i64 * MAX_MODES), ("n_hits", c_i32)]


class TkResult(ctypes.Structure):
    _fields_ = [("core", c_vp), ("factor", c_vp * MAX_MODES), ("ranks_eff", c_i32 * MAX_MODES),
                ("sweeps", c_i32), ("converged", c_i32), ("n_hits", c_i32),
                ("fit", c_dbl), ("err_model", c_dbl), ("norm_ytilde", c_dbl)]


class TkStats(ctypes.Structure):
    _fields_ = [("T", c_i64), ("T_committed", c_i64), ("blocks", c_i64), ("nodes", c_i64),
                ("merges_total", c_i64), ("merges_last", c_i64), ("store_bytes", c_i64),
                ("height", c_i32)]


# (name, restype, argtypes) of every entry point declared in include/tucket.h
SIGNATURES = [
    ("tk_create", c_i32, [ctypes.POINTER(TkConfig), c_vp, ctypes.POINTER(c_vp)]),
    ("tk_destroy", None, [c_vp]),
    ("tk_last_error", ctypes.c_char_p, [c_vp]),
    ("tk_append", c_i32, [c_vp, c_vp, c_i32]),
    ("tk_build", c_i32, [c_vp, c_vp, c_i64, c_i32]),
    ("tk_hitset", c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(TkHit), c_i32, ctypes.POINTER(c_i32)]),
    ("tk_query_shape", c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(TkShape)]),
    ("tk_query", c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(TkResult)]),
    ("tk_query_batch", c_i32, [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                               ctypes.POINTER(TkResult)]),
    ("tk_set_query_iters", c_i32, [c_vp, c_i32, c_dbl]),
    ("tk_last_query_kernel_ms", c_i32, [c_vp, ctypes.POINTER(c_dbl)]),
    ("tk_last_query_profile", c_i32, [c_vp, c_i32, ctypes.POINTER(c_dbl)]),
    ("tk_stats_get", c_i32, [c_vp, ctypes.POINTER(TkStats)]),
    ("tk_node_ranks", c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    ("tk_read_node", c_i32, [c_vp, c_i32, c_i64, c_vp, ctypes.POINTER(c_vp)]),
    ("tk_restore_begin", c_i32, [c_vp, c_i64]),
    ("tk_load_node", c_i32, [c_vp, c_i32, c_i64, c_vp, ctypes.POINTER(c_vp)]),
    ("tk_hitset_plan", c_i32, [ctypes.POINTER(TkConfig), c_i64, c_i64, c_i64, ctypes.POINTER(TkHit),
                               c_i32, ctypes.POINTER(c_i32)]),
    ("tk_effective_ranks", c_i32, [ctypes.POINTER(TkConfig), c_i64, ctypes.POINTER(c_i32)]),
    ("tk_version", ctypes.c_char_p, []),
]

_LIB = None


def lib():
    """Load libtucket.so (built in-tree by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtucket.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class TuckerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


def make_config(dims: Sequence[int], ranks: Sequence[int], leaf_len: int = 1,
                theta: Tuple[int, int] = (7, 10), max_iter: int = 20, tol: float = 0.01,
                capacity_T: int = 0, prec: int = TK_F32, mem_budget_bytes: int = 0) -> TkConfig:
    cfg = TkConfig()
    cfg.p = 1 + len(dims)
    for n, d in enumerate(dims, start=1):
        cfg.dims[n] = int(d)
    for n, r in enumerate(ranks):
        cfg.ranks[n] = int(r)
    cfg.leaf_len = int(leaf_len)
    cfg.theta_num, cfg.theta_den = int(theta[0]), int(theta[1])
    cfg.max_iter = int(max_iter)
    cfg.tol = float(tol)
    cfg.prec = int(prec)
    cfg.capacity_T = int(capacity_T)
    cfg.mem_budget_bytes = int(mem_budget_bytes)
    return cfg


def _hits_to_list(buf, n):
    return [dict(level=h.level, index=h.index, node_id=h.node_id, sigma=h.sigma, tau=h.tau,
                 lo=h.lo, hi=h.hi, partial=bool(h.partial)) for h in buf[:n]]


def hitset_plan(cfg: TkConfig, T: int, ts: int, te: int) -> List[dict]:
    """Host-only pruned hit set of [ts, te) for a tree of horizon T."""
    L = lib()
    n = c_i32(0)
    buf = (TkHit * 128)()
    st = L.tk_hitset_plan(ctypes.byref(cfg), T, ts, te, buf, 128, ctypes.byref(n))
    if st != TK_OK:
        raise TuckerError(st, "tk_hitset_plan")
    return _hits_to_list(buf, n.value)


def effective_ranks(cfg: TkConfig, length: int) -> Tuple[int, ...]:
    out = (c_i32 * MAX_MODES)()
    st = lib().tk_effective_ranks(ctypes.byref(cfg), length, out)
    if st != TK_OK:
        raise TuckerError(st, "tk_effective_ranks")
    return tuple(out[:cfg.p])


class QueryResult:
    """A range query's decomposition; tensors live on the device."""

    def __init__(self, core, factors, res: TkResult, p: int):
        self.core = core
        self.factors = factors
        self.ranks = tuple(res.ranks_eff[:p])
        self.sweeps = res.sweeps
        self.converged = bool(res.converged)
        self.n_hits = res.n_hits
        self.fit = res.fit
        self.err_model = res.err_model
        self.norm_ytilde = res.norm_ytilde


class PreparedBatch:
    """A list of range queries with device output buffers allocated once."""

    def __init__(self, tree: "Tree", ts, te):
        self.tree = tree
        self.ts = np.asarray(ts, dtype=np.int64).reshape(-1)
        self.te = np.asarray(te, dtype=np.int64).reshape(-1)
        n = len(self.ts)
        self.n = n
        p = tree.p
        shapes_all = []
        for i in range(n):
            sh = tree.query_shape(int(self.ts[i]), int(self.te[i]))
            r = tuple(sh.ranks_eff[:p])
            shapes_all.append([r, (int(self.te[i] - self.ts[i]), r[0])] +
                              [(tree.dims[m - 1], r[m]) for m in range(1, p)])
        self.buf, views = tree._alloc([s for shp in shapes_all for s in shp])
        self.res = (TkResult * max(n, 1))()
        self.outputs = []
        k = 0
        for i in range(n):
            core, facs = views[k], views[k + 1:k + 1 + p]
            k += 1 + p
            self.res[i].core = core.data_ptr()
            for m in range(p):
                self.res[i].factor[m] = facs[m].data_ptr()
            self.outputs.append((core, facs))
        self._ts = (c_i64 * max(n, 1))(*self.ts.tolist())
        self._te = (c_i64 * max(n, 1))(*self.te.tolist())

    def run(self):
        """One tk_query_batch call: Recall, trims and Stitch for every query."""
        self.tree._check(lib().tk_query_batch(self.tree._h, self.n, self._ts, self._te, self.res),
                         "tk_query_batch")

    def run_one(self, i: int):
        """Query i alone (one device launch)."""
        ts = ctypes.cast(ctypes.addressof(self._ts) + 8 * i, ctypes.POINTER(c_i64))
        te = ctypes.cast(ctypes.addressof(self._te) + 8 * i, ctypes.POINTER(c_i64))
        res = ctypes.cast(ctypes.addressof(self.res) + ctypes.sizeof(TkResult) * i, ctypes.POINTER(TkResult))
        self.tree._check(lib().tk_query_batch(self.tree._h, 1, ts, te, res), "tk_query")

    def results(self) -> List[QueryResult]:
        return [QueryResult(c, f, self.res[i], self.tree.p) for i, (c, f) in enumerate(self.outputs)]


class Tree:
    """A stream segment tree on the current HIP device."""

    def __init__(self, dims: Sequence[int], ranks: Sequence[int], leaf_len: int = 1,
                 theta: Tuple[int, int] = (7, 10), max_iter: int = 20, tol: float = 0.01,
                 capacity_T: int = 1 << 16, prec: int = TK_F32, mem_budget_bytes: int = 0,
                 stream=None):
        import torch
        self._torch = torch
        self.cfg = make_config(dims, ranks, leaf_len, theta, max_iter, tol, capacity_T, prec,
                               mem_budget_bytes)
        self.p = self.cfg.p
        self.dims = tuple(int(d) for d in dims)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_vp(0)
        st = lib().tk_create(ctypes.byref(self.cfg), c_vp(stream.cuda_stream), ctypes.byref(h))
        if st != TK_OK:
            raise TuckerError(st, lib().tk_last_error(None).decode())
        self._h = h

    # -- helpers -----------------------------------------------------------------
    def _check(self, st, what):
        if st != TK_OK:
            raise TuckerError(st, "%s: %s" % (what, lib().tk_last_error(self._h).decode()))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tk_destroy(self._h)
            self._h = c_vp(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _device_f32(self, X):
        torch = self._torch
        if isinstance(X, np.ndarray):
            X = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32))
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        return X

    # -- stream updates ------------------------------------------------------------
    def append(self, slice_):
        X = self._device_f32(slice_)
        assert tuple(X.shape) == self.dims, "slice shape %s != %s" % (tuple(X.shape), self.dims)
        self._check(lib().tk_append(self._h, c_vp(X.data_ptr()), 1), "tk_append")

    def build(self, X):
        X = self._device_f32(X)
        assert tuple(X.shape[1:]) == self.dims
        self._check(lib().tk_build(self._h, c_vp(X.data_ptr()), X.shape[0], 1), "tk_build")

    # -- queries ---------------------------------------------------------------------
    def hitset(self, ts: int, te: int) -> List[dict]:
        n = c_i32(0)
        buf = (TkHit * 128)()
        self._check(lib().tk_hitset(self._h, ts, te, buf, 128, ctypes.byref(n)), "tk_hitset")
        return _hits_to_list(buf, n.value)

    def query_shape(self, ts: int, te: int) -> TkShape:
        sh = TkShape()
        self._check(lib().tk_query_shape(self._h, ts, te, ctypes.byref(sh)), "tk_query_shape")
        return sh

    def _alloc(self, shapes):
        torch = self._torch
        total = sum(int(np.prod(s)) for s in shapes)
        buf = torch.empty(max(total, 1), dtype=torch.float32, device="cuda")
        views, off = [], 0
        for s in shapes:
            n = int(np.prod(s))
            views.append(buf[off:off + n].view(*s))
            off += n
        return buf, views

    def prepare_batch(self, ts, te) -> "PreparedBatch":
        """Allocate the outputs of a fixed list of queries once; run() reuses them."""
        return PreparedBatch(self, ts, te)

    def query_batch(self, ts, te) -> List[QueryResult]:
        b = self.prepare_batch(ts, te)
        b.run()
        return b.results()

    PHASES = ("trim", "basis", "init", "t_ttm_gram", "t_eig", "n_ttm_gram", "n_eig", "final")
    COUNTERS = ("eig_calls", "eig_sweeps", "eig_rot_us", "eig_tail_us")

    def last_profile(self, i: int) -> dict:
        out = (c_dbl * 12)()
        self._check(lib().tk_last_query_profile(self._h, i, out), "tk_last_query_profile")
        return dict(zip(self.PHASES + self.COUNTERS, list(out)))

    def last_kernel_ms(self) -> float:
        ms = c_dbl(0.0)
        self._check(lib().tk_last_query_kernel_ms(self._h, ctypes.byref(ms)), "tk_last_query_kernel_ms")
        return ms.value

    def query(self, ts: int, te: int) -> QueryResult:
        return self.query_batch([ts], [te])[0]

    def set_query_iters(self, max_iter: int, tol: float):
        self._check(lib().tk_set_query_iters(self._h, max_iter, tol), "tk_set_query_iters")

    # -- store access ---------------------------------------------------------------------
    def stats(self) -> dict:
        s = TkStats()
        self._check(lib().tk_stats_get(self._h, ctypes.byref(s)), "tk_stats_get")
        return {k: getattr(s, k) for k, _ in TkStats._fields_}

    def node_ranks(self, level: int) -> Tuple[int, ...]:
        out = (c_i32 * MAX_MODES)()
        self._check(lib().tk_node_ranks(self._h, level, out), "tk_node_ranks")
        return tuple(out[:self.p])

    def _node_shapes(self, level):
        r = self.node_ranks(level)
        rows = self.cfg.leaf_len << level
        return r, [(rows, r[0])] + [(self.dims[m - 1], r[m]) for m in range(1, self.p)]

    def read_node(self, level: int, index: int):
        r, fshapes = self._node_shapes(level)
        core = np.empty(r, dtype=np.float32)
        facs = [np.empty(s, dtype=np.float32) for s in fshapes]
        ptrs = (c_vp * MAX_MODES)(*[f.ctypes.data for f in facs])
        self._check(lib().tk_read_node(self._h, level, index, c_vp(core.ctypes.data), ptrs),
                    "tk_read_node")
        return core, facs

    def restore_begin(self, T: int):
        self._check(lib().tk_restore_begin(self._h, T), "tk_restore_begin")

    def load_node(self, level: int, index: int, core, factors):
        r, fshapes = self._node_shapes(level)
        core = np.ascontiguousarray(core, dtype=np.float32).reshape(r)
        facs = [np.ascontiguousarray(f, dtype=np.float32).reshape(s) for f, s in zip(factors, fshapes)]
        ptrs = (c_vp * MAX_MODES)(*[f.ctypes.data for f in facs])
        self._check(lib().tk_load_node(self._h, level, index, c_vp(core.ctypes.data), ptrs),
                    "tk_load_node")
