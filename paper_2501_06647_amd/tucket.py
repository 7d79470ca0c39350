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
LIB_PATH = os.environ.get("TUCKET_LIB") or os.path.join(_HERE, "libtucket.so")
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
                ("factor_elems", c_i64 * MAX_MODES), ("n_hits", c_i32), ("ws_bytes", c_i64)]


class TkResult(ctypes.Structure):
    _fields_ = [("core", c_vp), ("factor", c_vp * MAX_MODES), ("ranks_eff", c_i32 * MAX_MODES),
                ("sweeps", c_i32), ("converged", c_i32), ("n_hits", c_i32),
                ("fit", c_dbl), ("err_model", c_dbl), ("norm_ytilde", c_dbl)]


class TkStats(ctypes.Structure):
    _fields_ = [("T", c_i64), ("T_committed", c_i64), ("blocks", c_i64), ("nodes", c_i64),
                ("merges_total", c_i64), ("merges_last", c_i64), ("store_bytes", c_i64),
                ("height", c_i32)]


class TkTuning(ctypes.Structure):
    _fields_ = [("wide_threshold", c_i32), ("wide_threads", c_i32), ("persistent", c_i32), ("graph", c_i32),
                ("coarse", c_i32), ("lds_n", c_i32), ("basis_pct", c_i32),
                ("rest_threads", c_i32), ("wide_core", c_i32)]


class TkServeConfig(ctypes.Structure):
    _fields_ = [("max_batch", c_i32), ("max_commit_blocks", c_i32), ("ws_budget_bytes", c_i64),
                ("max_queue", c_i64)]


class TkServeStats(ctypes.Structure):
    _fields_ = [("queries", c_i64), ("appends", c_i64), ("completed", c_i64), ("rejected", c_i64),
                ("batches", c_i64), ("commits", c_i64), ("max_batch_seen", c_i64), ("outstanding", c_i64),
                ("T_submitted", c_i64), ("T_committed", c_i64)]


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
    ("tk_query_noalloc", c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(TkResult)]),
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
    ("tk_set_query_prec", c_i32, [c_vp, c_i32]),
    ("tk_set_query_ranks", c_i32, [c_vp, c_vp]),
    ("tk_set_query_recall", c_i32, [c_vp, c_i32]),
    ("tk_raw_tucker", c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    ("tk_raw_tucker_stream", c_i32, [c_vp, c_vp, c_i64, c_vp]),
    ("tk_get_tuning", c_i32, [c_vp, ctypes.POINTER(TkTuning)]),
    ("tk_set_tuning", c_i32, [c_vp, ctypes.POINTER(TkTuning)]),
    ("tk_batch_create", c_i32, [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                ctypes.POINTER(TkResult), ctypes.POINTER(c_vp)]),
    ("tk_batch_run", c_i32, [c_vp]),
    ("tk_batch_wait", c_i32, [c_vp]),
    ("tk_batch_kernel_ms", c_i32, [c_vp, ctypes.POINTER(c_dbl)]),
    ("tk_batch_profile", c_i32, [c_vp, c_i32, ctypes.POINTER(c_dbl)]),
    ("tk_batch_hits", c_i32, [c_vp, c_i32, ctypes.POINTER(TkHit), c_i32, ctypes.POINTER(c_i32)]),
    ("tk_batch_destroy", None, [c_vp]),
    ("tk_set_autotune_limits", c_i32, [c_vp, c_dbl, c_dbl, c_i32]),
    ("tk_autotune", c_i32, [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_i32,
                            ctypes.POINTER(TkTuning), ctypes.POINTER(c_dbl)]),
    ("tk_serve_start", c_i32, [c_vp, ctypes.POINTER(TkServeConfig)]),
    ("tk_serve_stop", c_i32, [c_vp]),
    ("tk_submit_query", c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(TkResult), ctypes.POINTER(ctypes.c_uint64)]),
    ("tk_submit_append", c_i32, [c_vp, c_vp, c_i32, ctypes.POINTER(ctypes.c_uint64)]),
    ("tk_poll", c_i32, [c_vp, ctypes.c_uint64, ctypes.POINTER(c_i32)]),
    ("tk_wait", c_i32, [c_vp, ctypes.c_uint64]),
    ("tk_sync", c_i32, [c_vp]),
    ("tk_ticket_times", c_i32, [c_vp, ctypes.c_uint64, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                                ctypes.POINTER(c_dbl)]),
    ("tk_serve_stats_get", c_i32, [c_vp, ctypes.POINTER(TkServeStats)]),
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


def _query_shapes(tree, ts, te):
    """Output shapes of each query: core, U^(1), U^(2..p).  An empty or
    negative range raises TK_ERANGE here; a range past the committed horizon
    is refused by the library call that takes it."""
    p = tree.p
    out = []
    for a, b in zip(ts, te):
        if not (0 <= int(a) < int(b)):
            raise TuckerError(TK_ERANGE, "query range [%d, %d) is empty or negative" % (int(a), int(b)))
        r = effective_ranks(tree.query_cfg(), int(b - a))
        out.append([r, (int(b - a), r[0])] + [(tree.dims[m - 1], r[m]) for m in range(1, p)])
    return out


class PreparedBatch:
    """A fixed list of range queries planned once (tk_batch_create): device
    outputs allocated once, job descriptors resident, launches captured in a
    HIP graph when the tree's tuning asks for it.  Every run() executes
    Recall, trims and Stitch of every query on the device."""

    def __init__(self, tree: "Tree", ts, te):
        self.tree = tree
        self.ts = np.asarray(ts, dtype=np.int64).reshape(-1)
        self.te = np.asarray(te, dtype=np.int64).reshape(-1)
        n = len(self.ts)
        self.n = n
        p = tree.p
        shapes_all = _query_shapes(tree, self.ts, self.te)
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
        self._h = c_vp(0)
        if n > 0:
            tree._check(lib().tk_batch_create(tree._h, n, self._ts, self._te, self.res, ctypes.byref(self._h)),
                        "tk_batch_create")

    def run(self, wait: bool = True):
        """One execution on the tree's stream (graph replay); with wait, block
        and collect the per-query scalars."""
        if self.n == 0:
            return
        self.tree._check(lib().tk_batch_run(self._h), "tk_batch_run")
        if wait:
            self.wait()

    def wait(self):
        self.tree._check(lib().tk_batch_wait(self._h), "tk_batch_wait")

    def run_sync(self):
        """The same queries through tk_query_batch: host Recall and planning,
        then the launches, every call."""
        self.tree._check(lib().tk_query_batch(self.tree._h, self.n, self._ts, self._te, self.res),
                         "tk_query_batch")

    def run_one(self, i: int):
        """Query i alone (one device launch)."""
        ts = ctypes.cast(ctypes.addressof(self._ts) + 8 * i, ctypes.POINTER(c_i64))
        te = ctypes.cast(ctypes.addressof(self._te) + 8 * i, ctypes.POINTER(c_i64))
        res = ctypes.cast(ctypes.addressof(self.res) + ctypes.sizeof(TkResult) * i, ctypes.POINTER(TkResult))
        self.tree._check(lib().tk_query_batch(self.tree._h, 1, ts, te, res), "tk_query")

    def kernel_ms(self) -> float:
        ms = c_dbl(0.0)
        self.tree._check(lib().tk_batch_kernel_ms(self._h, ctypes.byref(ms)), "tk_batch_kernel_ms")
        return ms.value

    def profile(self, i: int) -> dict:
        out = (c_dbl * len(Tree.PHASES + Tree.COUNTERS))()
        self.tree._check(lib().tk_batch_profile(self._h, i, out), "tk_batch_profile")
        return dict(zip(Tree.PHASES + Tree.COUNTERS, list(out)))

    def device_hits(self, i: int) -> List[dict]:
        """The hit set query i's kernel computed on the device."""
        n = c_i32(0)
        buf = (TkHit * 128)()
        self.tree._check(lib().tk_batch_hits(self._h, i, buf, 128, ctypes.byref(n)), "tk_batch_hits")
        return _hits_to_list(buf, n.value)

    def results(self) -> List[QueryResult]:
        return [QueryResult(c, f, self.res[i], self.tree.p) for i, (c, f) in enumerate(self.outputs)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tk_batch_destroy(self._h)
            self._h = c_vp(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop of a tree (tk_serve_start): queries
    and appends are submitted and return tickets; results are read once a
    ticket is done.  Output buffers are allocated per query on the device
    and kept until the result is taken."""

    def __init__(self, tree: "Tree", max_batch: int = 0, max_commit_blocks: int = 0,
                 ws_budget_bytes: int = 0, max_queue: int = 0):
        self.tree = tree
        cfg = TkServeConfig(int(max_batch), int(max_commit_blocks), int(ws_budget_bytes), int(max_queue))
        tree._check(lib().tk_serve_start(tree._h, ctypes.byref(cfg)), "tk_serve_start")
        self._live = {}
        self.running = True

    def submit_query(self, ts: int, te: int) -> int:
        tree = self.tree
        shp = _query_shapes(tree, [ts], [te])[0]
        buf, views = tree._alloc(shp)
        res = TkResult()
        res.core = views[0].data_ptr()
        for m in range(tree.p):
            res.factor[m] = views[1 + m].data_ptr()
        t = ctypes.c_uint64(0)
        tree._check(lib().tk_submit_query(tree._h, int(ts), int(te), ctypes.byref(res), ctypes.byref(t)),
                    "tk_submit_query")
        self._live[t.value] = (res, buf, views)
        return t.value

    def submit_append(self, slice_) -> int:
        tree = self.tree
        t = ctypes.c_uint64(0)
        if isinstance(slice_, np.ndarray):
            x = np.ascontiguousarray(slice_, dtype=np.float32)
            assert x.shape == tree.dims
            tree._check(lib().tk_submit_append(tree._h, c_vp(x.ctypes.data), 0, ctypes.byref(t)),
                        "tk_submit_append")
        else:
            x = tree._device_f32(slice_)
            assert tuple(x.shape) == tree.dims
            tree._check(lib().tk_submit_append(tree._h, c_vp(x.data_ptr()), 1, ctypes.byref(t)),
                        "tk_submit_append")
            self._live[t.value] = (None, x, None)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = c_i32(0)
        self.tree._check(lib().tk_poll(self.tree._h, ticket, ctypes.byref(d)), "tk_poll")
        return bool(d.value)

    def wait(self, ticket: int):
        self.tree._check(lib().tk_wait(self.tree._h, ticket), "tk_wait")

    def sync(self):
        self.tree._check(lib().tk_sync(self.tree._h), "tk_sync")

    def result(self, ticket: int) -> QueryResult:
        """The decomposition of a finished query (releases the ticket's buffers)."""
        self.wait(ticket)
        res, buf, views = self._live.pop(ticket)
        return QueryResult(views[0], views[1:], res, self.tree.p)

    def release(self, ticket: int):
        self._live.pop(ticket, None)

    def times(self, ticket: int) -> Tuple[float, float, float]:
        a, b, c = c_dbl(), c_dbl(), c_dbl()
        self.tree._check(lib().tk_ticket_times(self.tree._h, ticket, ctypes.byref(a), ctypes.byref(b),
                                               ctypes.byref(c)), "tk_ticket_times")
        return a.value, b.value, c.value

    def stats(self) -> dict:
        s = TkServeStats()
        self.tree._check(lib().tk_serve_stats_get(self.tree._h, ctypes.byref(s)), "tk_serve_stats_get")
        return {k: getattr(s, k) for k, _ in TkServeStats._fields_}

    def stop(self):
        if self.running:
            self.running = False
            self.tree._check(lib().tk_serve_stop(self.tree._h), "tk_serve_stop")
            self._live.clear()


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
        """Plan a fixed list of queries once; run() replays them."""
        return PreparedBatch(self, ts, te)

    def raw_tucker(self, X, ts, te) -> List[QueryResult]:
        """tk_raw_tucker: Tucker-ALS from scratch on the ranges [ts_i, te_i)
        of the series X (T x D_2 x ... x D_p; moved to the device if it is
        not there), at the query output ranks."""
        X = self._device_f32(X)
        assert tuple(X.shape[1:]) == self.dims
        ts = np.asarray(ts, dtype=np.int64).reshape(-1)
        te = np.asarray(te, dtype=np.int64).reshape(-1)
        n = len(ts)
        if n and (te.max() > X.shape[0] or ts.min() < 0):
            raise TuckerError(TK_ERANGE, "raw range outside the series")
        p = self.p
        shapes_all = _query_shapes(self, ts, te)
        buf, views = self._alloc([s for shp in shapes_all for s in shp])
        res = (TkResult * max(n, 1))()
        outputs = []
        k = 0
        for i in range(n):
            core, facs = views[k], views[k + 1:k + 1 + p]
            k += 1 + p
            res[i].core = core.data_ptr()
            for m in range(p):
                res[i].factor[m] = facs[m].data_ptr()
            outputs.append((core, facs))
        slice_bytes = int(np.prod(self.dims)) * 4
        ptrs = (c_vp * max(n, 1))(*[X.data_ptr() + int(a) * slice_bytes for a in ts])
        lens = (c_i64 * max(n, 1))(*(te - ts).tolist())
        if n:
            self._check(lib().tk_raw_tucker(self._h, n, ptrs, lens, res), "tk_raw_tucker")
        return [QueryResult(c, f, res[i], p) for i, (c, f) in enumerate(outputs)]

    def raw_tucker_stream(self, X, ts, te) -> QueryResult:
        """tk_raw_tucker_stream: Tucker-ALS from scratch on the range
        [ts, te) of the series X (on the device, or moved there) with many
        workgroups per pass."""
        X = self._device_f32(X)
        assert tuple(X.shape[1:]) == self.dims
        ts, te = int(ts), int(te)
        if not (0 <= ts < te <= X.shape[0]):
            raise TuckerError(TK_ERANGE, "raw range outside the series")
        p = self.p
        shapes = _query_shapes(self, np.array([ts], dtype=np.int64), np.array([te], dtype=np.int64))[0]
        buf, views = self._alloc(shapes)
        core, facs = views[0], views[1:1 + p]
        res = TkResult()
        res.core = core.data_ptr()
        for m in range(p):
            res.factor[m] = facs[m].data_ptr()
        slice_bytes = int(np.prod(self.dims)) * 4
        self._check(lib().tk_raw_tucker_stream(self._h, X.data_ptr() + ts * slice_bytes, te - ts, ctypes.byref(res)),
                    "tk_raw_tucker_stream")
        return QueryResult(core, facs, res, p)

    def query_batch(self, ts, te) -> List[QueryResult]:
        """tk_query_batch: one synchronous batched call (host Recall and
        planning every call; a range may end in the incomplete block)."""
        ts = np.asarray(ts, dtype=np.int64).reshape(-1)
        te = np.asarray(te, dtype=np.int64).reshape(-1)
        n = len(ts)
        p = self.p
        shapes_all = _query_shapes(self, ts, te)
        buf, views = self._alloc([s for shp in shapes_all for s in shp])
        res = (TkResult * max(n, 1))()
        outputs = []
        k = 0
        for i in range(n):
            core, facs = views[k], views[k + 1:k + 1 + p]
            k += 1 + p
            res[i].core = core.data_ptr()
            for m in range(p):
                res[i].factor[m] = facs[m].data_ptr()
            outputs.append((core, facs))
        a = (c_i64 * max(n, 1))(*ts.tolist())
        b = (c_i64 * max(n, 1))(*te.tolist())
        if n:
            self._check(lib().tk_query_batch(self._h, n, a, b, res), "tk_query_batch")
        return [QueryResult(c, f, res[i], p) for i, (c, f) in enumerate(outputs)]

    # -- launch tuning and serving -----------------------------------------------------
    def tuning(self) -> dict:
        tu = TkTuning()
        self._check(lib().tk_get_tuning(self._h, ctypes.byref(tu)), "tk_get_tuning")
        return {k: getattr(tu, k) for k, _ in TkTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        tu = TkTuning(**{k: int(v) for k, v in cur.items()})
        self._check(lib().tk_set_tuning(self._h, ctypes.byref(tu)), "tk_set_tuning")

    def autotune(self, ts, te, reps: int = 2, budget_s: float = 60.0, cap: float = 3.0,
                 progress: bool = False) -> Tuple[dict, float]:
        """Search launch tunings on these queries (tk_autotune) within a
        time budget, abandoning candidates whose warm-up exceeds cap x the
        best so far; progress: one stderr line per candidate."""
        self._check(lib().tk_set_autotune_limits(self._h, float(budget_s), float(cap), int(bool(progress))),
                    "tk_set_autotune_limits")
        ts = np.asarray(ts, dtype=np.int64).reshape(-1)
        te = np.asarray(te, dtype=np.int64).reshape(-1)
        n = len(ts)
        a = (c_i64 * n)(*ts.tolist())
        b = (c_i64 * n)(*te.tolist())
        tu = TkTuning()
        ms = c_dbl(0.0)
        self._check(lib().tk_autotune(self._h, n, a, b, reps, ctypes.byref(tu), ctypes.byref(ms)), "tk_autotune")
        return {k: getattr(tu, k) for k, _ in TkTuning._fields_}, ms.value

    def serve(self, **kw) -> "Server":
        return Server(self, **kw)

    PHASES = ("trim", "basis", "init", "t_ttm_gram", "t_eig", "n_ttm_gram", "n_eig", "final")
    COUNTERS = ("eig_calls", "eig_bisect_steps", "eig_values_us", "eig_vectors_us", "start_us", "end_us",
                "eig_fallbacks", "eig_tridiag_us", "eig_invit_us", "eig_warm", "eig_warm_refused",
                "eig_warm_steps", "eig_warm_us", "eig_warm_rr_us")

    def last_profile(self, i: int) -> dict:
        out = (c_dbl * len(Tree.PHASES + Tree.COUNTERS))()
        self._check(lib().tk_last_query_profile(self._h, i, out), "tk_last_query_profile")
        return dict(zip(self.PHASES + self.COUNTERS, list(out)))

    def last_kernel_ms(self) -> float:
        ms = c_dbl(0.0)
        self._check(lib().tk_last_query_kernel_ms(self._h, ctypes.byref(ms)), "tk_last_query_kernel_ms")
        return ms.value

    def query(self, ts: int, te: int) -> QueryResult:
        return self.query_batch([ts], [te])[0]

    def query_noalloc(self, ts: int, te: int, out: Optional[QueryResult] = None) -> QueryResult:
        """tk_query_noalloc: the library allocates nothing (its fixed device
        scratch); the outputs are the caller's (``out``'s buffers when
        given, else new ones)."""
        if out is None:
            shp = _query_shapes(self, [ts], [te])[0]
            _, views = self._alloc(shp)
            core, facs = views[0], views[1:]
        else:
            core, facs = out.core, out.factors
        res = TkResult()
        res.core = core.data_ptr()
        for m in range(self.p):
            res.factor[m] = facs[m].data_ptr()
        self._check(lib().tk_query_noalloc(self._h, int(ts), int(te), ctypes.byref(res)), "tk_query_noalloc")
        return QueryResult(core, list(facs), res, self.p)

    def set_query_iters(self, max_iter: int, tol: float):
        self._check(lib().tk_set_query_iters(self._h, max_iter, tol), "tk_set_query_iters")

    def set_query_prec(self, prec: int):
        """TK_F32 or TK_BF16 arithmetic for later queries."""
        self._check(lib().tk_set_query_prec(self._h, int(prec)), "tk_set_query_prec")

    def set_query_ranks(self, ranks=None):
        """Output ranks r_1..r_p of later queries (each at most the node
        rank); None restores the tree's ranks."""
        if ranks is None:
            arg = None
        else:
            arg = (c_i32 * MAX_MODES)(*[int(r) for r in ranks])
        self._check(lib().tk_set_query_ranks(self._h, arg), "tk_set_query_ranks")
        self._q_ranks = None if ranks is None else tuple(int(r) for r in ranks)

    def set_query_recall(self, level=None):
        """Hit sets of later queries: None for Alg. "recall", or the
        fixed-block variant at that tree level."""
        self._check(lib().tk_set_query_recall(self._h, -1 if level is None else int(level)),
                    "tk_set_query_recall")

    def query_cfg(self) -> TkConfig:
        """The tree's config with the query output ranks in place of its ranks."""
        q = getattr(self, "_q_ranks", None)
        if q is None:
            return self.cfg
        c = TkConfig()
        ctypes.pointer(c)[0] = self.cfg
        for n, r in enumerate(q):
            c.ranks[n] = r
        return c

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
