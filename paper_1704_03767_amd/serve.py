"""Python binding of the query-vs-database path and the query server of
libktau (include/ktau.h): argument marshalling only.

``KtauDb`` ranks a database once into HBM (ktau_db_create); ``ktau_query``
runs one stream-ordered query launch; ``KtauServer`` wraps the library's
continuous-batching server (ktau_server_*), whose worker thread admits,
merges and launches requests inside the library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .ktau import KTAU_OK, KtauError, _as_matrix, _check, _ptr, _stream, lib, scheme_id

KTAU_MAX_K = 1024


class _ServerCfg(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch_queries", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_int64), ("max_queue", ctypes.c_int32),
                ("k_max", ctypes.c_int32)]


class Latency(ctypes.Structure):
    _fields_ = [("queue_us", ctypes.c_double), ("device_us", ctypes.c_double),
                ("total_us", ctypes.c_double), ("batch_queries", ctypes.c_int64),
                ("batch_requests", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("launches", "merged_requests", "completed",
                                              "failed", "peak_pool_bytes", "peak_running",
                                              "queued")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _slib():
    L = lib()
    if getattr(L, "_ktau_serve_declared", False):
        return L
    i64, i32, p, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    decl = {
        "ktau_db_create": ([p, i64, i64, p, p], i32),
        "ktau_db_create_ex": ([p, i64, i64, i32, p, p], i32),
        "ktau_db_destroy": ([p], None),
        "ktau_db_rows": ([p], i64),
        "ktau_db_samples": ([p], i64),
        "ktau_query_workspace_size": ([p, i64, i64], sz),
        "ktau_query": ([p, p, i64, i64, p, p, p, p, sz, p], i32),
        "ktau_server_default_cfg": ([p], None),
        "ktau_server_create": ([p, p, p], i32),
        "ktau_server_submit": ([p, p, i64, i64, i32, p], i32),
        "ktau_server_wait": ([p, i64, p, p, p, p, i64], i32),
        "ktau_server_cancel": ([p, i64], i32),
        "ktau_server_inject_failure": ([p, i64], i32),
        "ktau_server_stats": ([p, p], i32),
        "ktau_server_pause": ([p, i32], i32),
        "ktau_server_destroy": ([p], None),
        "ktau_server_launch_bytes": ([p, i64, i64], sz),
        "ktau_status": ([p, p], i32),
    }
    for name, (args, res) in decl.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    L._ktau_serve_declared = True
    return L


class KtauDb:
    """A database ranked once and kept resident in HBM (ktau_db_create; with
    ``scheme`` given, ktau_db_create_ex and that network scheme)."""

    def __init__(self, X: torch.Tensor, stream=None, scheme=None):
        X = _as_matrix(X)
        h = ctypes.c_void_p()
        if scheme is None:
            _check(_slib().ktau_db_create(_ptr(X), X.shape[0], X.shape[1], _stream(stream),
                                          ctypes.byref(h)), "ktau_db_create")
        else:
            _check(_slib().ktau_db_create_ex(_ptr(X), X.shape[0], X.shape[1], scheme_id(scheme),
                                             _stream(stream), ctypes.byref(h)),
                   "ktau_db_create_ex")
        self._h = h
        self.m, self.n = X.shape

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _slib().ktau_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ktau_query_workspace_size(db: KtauDb, nq: int, k: int) -> int:
    return int(_slib().ktau_query_workspace_size(db.handle, nq, k))


def ktau_query(db: KtauDb, Q: torch.Tensor, k: int, workspace: torch.Tensor | None = None,
               stream=None, check: bool = True) -> dict:
    """Top-k database rows by |tau_B| for every row of Q (a CUDA float32
    nq x n tensor).  Returns device tensors idx (int64), tau (float64), nd
    (int64), each nq x k."""
    Q = _as_matrix(Q)
    nq = Q.shape[0]
    dev = Q.device
    idx = torch.empty((nq, k), dtype=torch.int64, device=dev)
    tau = torch.empty((nq, k), dtype=torch.float64, device=dev)
    nd = torch.empty((nq, k), dtype=torch.int64, device=dev)
    if workspace is None:
        size = ktau_query_workspace_size(db, nq, k)
        if size == 0:
            raise KtauError(-1, "ktau_query_workspace_size")
        workspace = torch.empty(size, dtype=torch.uint8, device=dev)
    _check(_slib().ktau_query(db.handle, _ptr(Q), nq, k, _ptr(idx), _ptr(tau), _ptr(nd),
                              _ptr(workspace), workspace.numel(), _stream(stream)), "ktau_query")
    if check:
        st = int(_slib().ktau_status(_ptr(workspace), _stream(stream)))
        if st != KTAU_OK:
            raise KtauError(st, "ktau_query")
    return {"idx": idx, "tau": tau, "nd": nd}


class KtauServer:
    """The library's continuous-batching query server over a KtauDb."""

    def __init__(self, db: KtauDb, slots: int = 2, max_batch_queries: int = 256,
                 mem_budget_bytes: int = 1 << 30, max_queue: int = 4096, k_max: int = 128):
        L = _slib()
        cfg = _ServerCfg()
        L.ktau_server_default_cfg(ctypes.byref(cfg))
        cfg.slots, cfg.max_batch_queries = slots, max_batch_queries
        cfg.mem_budget_bytes, cfg.max_queue, cfg.k_max = mem_budget_bytes, max_queue, k_max
        h = ctypes.c_void_p()
        _check(L.ktau_server_create(db.handle, ctypes.byref(cfg), ctypes.byref(h)),
               "ktau_server_create")
        self._h = h
        self.db = db
        self._k = {}

    def submit(self, q: np.ndarray, k: int, blocking: bool = True) -> int:
        """Queues the rows of q (host float32, nq x n); returns a ticket."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        if q.ndim == 1:
            q = q[None, :]
        t = ctypes.c_int64()
        _check(_slib().ktau_server_submit(self._h, ctypes.c_void_p(q.ctypes.data), q.shape[0], k,
                                          1 if blocking else 0, ctypes.byref(t)),
               "ktau_server_submit")
        self._k[t.value] = (q.shape[0], k)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(status, results dict or None, latency dict)."""
        nq, k = self._k[ticket]
        idx = np.empty((nq, k), np.int64)
        tau = np.empty((nq, k), np.float64)
        nd = np.empty((nq, k), np.int64)
        lat = Latency()
        st = int(_slib().ktau_server_wait(self._h, ticket, ctypes.c_void_p(idx.ctypes.data),
                                          ctypes.c_void_p(tau.ctypes.data),
                                          ctypes.c_void_p(nd.ctypes.data), ctypes.byref(lat),
                                          timeout_ms))
        if st == -8:   # still pending: the ticket stays valid
            return st, None, None
        del self._k[ticket]
        res = {"idx": idx, "tau": tau, "nd": nd} if st == KTAU_OK else None
        return st, res, lat.as_dict()

    def cancel(self, ticket: int) -> int:
        return int(_slib().ktau_server_cancel(self._h, ticket))

    def inject_failure(self, ticket: int) -> int:
        return int(_slib().ktau_server_inject_failure(self._h, ticket))

    def pause(self, paused: bool = True) -> None:
        """Stops or resumes admission of queued requests (ktau_server_pause)."""
        _check(_slib().ktau_server_pause(self._h, 1 if paused else 0), "ktau_server_pause")

    def stats(self) -> dict:
        c = Counters()
        _check(_slib().ktau_server_stats(self._h, ctypes.byref(c)), "ktau_server_stats")
        return c.as_dict()

    def launch_bytes(self, nq: int, k: int) -> int:
        """Device pool bytes of one launch of nq rows (ktau_server_launch_bytes)."""
        return int(_slib().ktau_server_launch_bytes(self._h, nq, k))

    def close(self):
        if getattr(self, "_h", None):
            _slib().ktau_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
