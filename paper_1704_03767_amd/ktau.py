"""Python binding of libktau (include/ktau.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  PyTorch
supplies device memory and the current HIP stream; all arithmetic of the
method runs in the HIP kernels of libktau.so.  If the library is not built,
every call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libktau.so")

KTAU_OK = 0
KTAU_EINVAL = -1
KTAU_ERANGE = -2
KTAU_ENOMEM = -3
KTAU_EDEVICE = -4
KTAU_EBUSY = -5
KTAU_ENAN = -6
KTAU_ECANCELED = -7
KTAU_ETIMEDOUT = -8
KTAU_MAX_N = 65536
KTAU_MAX_N_NETWORK = 32768     # query search and permutation test
KTAU_SCHEME_NAIVE = 100       # naive bit-set count, plain calls, n <= 256
NAIVE_SCHEME_NAME = "naive_bits"

_lock = threading.Lock()
_lib = None


class KtauError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class _PairOut(ctypes.Structure):
    _fields_ = [
        ("nc", ctypes.c_void_p), ("nd", ctypes.c_void_p), ("n3", ctypes.c_void_p),
        ("tau_b", ctypes.c_void_p), ("tau_a", ctypes.c_void_p), ("n1", ctypes.c_void_p),
    ]


def _declare(lib):
    i64, i32, p, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    decl = {
        "ktau_status_string": ([i32], ctypes.c_char_p),
        "ktau_pair_to_job": ([i64, i64, i64], i64),
        "ktau_job_to_pair": ([i64, i64, p, p], i32),
        "ktau_tile_to_coord": ([i64, i64, p, p], i32),
        "ktau_rank": ([p, i64, i64, p, p, p, p, p, p, sz, p], i32),
        "ktau_rank_workspace_size": ([i64, i64], sz),
        "ktau_allpairs_workspace_size": ([i64, i64], sz),
        "ktau_allpairs": ([p, i64, i64, _PairOut, p, sz, p], i32),
        "ktau_allpairs_noalloc": ([p, i64, i64, _PairOut, p, p], i32),
        "ktau_allpairs_range": ([p, i64, i64, i64, i64, _PairOut, p, sz, p], i32),
        "ktau_allpairs_ex": ([p, i64, i64, i64, i64, _PairOut, p, sz, i32, i32, p], i32),
        "ktau_status": ([p, p], i32),
        "ktau_prepare": ([p, i64, i64, p, p, sz, p], i32),
        "ktau_pairs": ([i64, i64, i64, i64, _PairOut, p, sz, i32, i32, p], i32),
        "ktau_scheme_count": ([], i32),
        "ktau_scheme_name": ([i32], ctypes.c_char_p),
        "ktau_scheme_capacity": ([i32], i64),
        "ktau_default_scheme": ([i64], i32),
        "ktau_plain_default_scheme": ([i64], i32),
        "ktau_plain_default_q": ([i64, i64], i32),
        "ktau_perm_workspace_size": ([i64, i64, i64], sz),
        "ktau_probe_threads": ([], i32),
        "ktau_probe_valu_ops_per_iter": ([], i32),
        "ktau_probe_lds_bytes_per_iter": ([], i32),
        "ktau_probe_valu": ([p, i64, i32, p], i32),
        "ktau_probe_issue": ([p, i64, i32, i32, p], i32),
        "ktau_probe_issue_instrs_per_iter": ([i32], i32),
        "ktau_probe_lds": ([p, i64, i32, p], i32),
        "ktau_perm_test": ([p, i64, i64, p, i64, i64, i64, p, p, p, sz, p], i32),
    }
    for name, (args, res) in decl.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


def lib():
    """The loaded libktau.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with `python -m paper_1704_03767_amd.build`")
            _lib = _declare(ctypes.CDLL(LIB_PATH))
        return _lib


def status_string(status: int) -> str:
    try:
        return lib().ktau_status_string(int(status)).decode()
    except RuntimeError:
        return "library not loaded"


def _check(rc: int, what: str):
    if rc != KTAU_OK:
        raise KtauError(rc, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _as_matrix(X: torch.Tensor) -> torch.Tensor:
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
        raise TypeError("X must be a CUDA (HIP) tensor")
    if X.dtype != torch.float32 or X.dim() != 2:
        raise TypeError("X must be a 2-D float32 tensor")
    return X.contiguous()


# ------------------------------------------------------------------ mapper


def ktau_pair_to_job(m: int, y: int, x: int) -> int:
    return int(lib().ktau_pair_to_job(m, y, x))


def ktau_job_to_pair(m: int, J: int) -> tuple[int, int]:
    y, x = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ktau_job_to_pair(m, J, ctypes.byref(y), ctypes.byref(x)), "ktau_job_to_pair")
    return y.value, x.value


def ktau_tile_to_coord(w: int, t: int) -> tuple[int, int]:
    y, x = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ktau_tile_to_coord(w, t, ctypes.byref(y), ctypes.byref(x)), "ktau_tile_to_coord")
    return y.value, x.value


def ktau_scheme_names() -> list[str]:
    L = lib()
    return [L.ktau_scheme_name(i).decode() for i in range(L.ktau_scheme_count())]


def ktau_scheme_capacity(scheme: int) -> int:
    return int(lib().ktau_scheme_capacity(int(scheme)))


def ktau_default_scheme(n: int) -> int:
    return int(lib().ktau_default_scheme(int(n)))


def ktau_plain_default_scheme(n: int) -> int:
    return int(lib().ktau_plain_default_scheme(int(n)))


def ktau_plain_default_q(m: int, n: int) -> int:
    return int(lib().ktau_plain_default_q(int(m), int(n)))


def scheme_name(scheme: int) -> str:
    """Name of a scheme id (a numbered scheme or KTAU_SCHEME_NAIVE)."""
    if int(scheme) == KTAU_SCHEME_NAIVE:
        return NAIVE_SCHEME_NAME
    return ktau_scheme_names()[int(scheme)]


def scheme_id(scheme) -> int:
    if scheme is None:
        return -1
    if isinstance(scheme, str):
        if scheme == NAIVE_SCHEME_NAME:
            return KTAU_SCHEME_NAIVE
        return ktau_scheme_names().index(scheme)
    return int(scheme)


# --------------------------------------------------------------- pre-pass


def ktau_rank(X: torch.Tensor, stream=None, check: bool = True) -> dict:
    """Per-row order, dense ranks, run starts (uint16 stored in int32 views)
    and n1, from the rank pre-pass kernel."""
    X = _as_matrix(X)
    m, n = X.shape
    dev = X.device
    perm = torch.empty((m, n), dtype=torch.int16, device=dev)
    rank = torch.empty((m, n), dtype=torch.int16, device=dev)
    rstart = torch.empty((m, n), dtype=torch.int16, device=dev)
    n1 = torch.empty(m, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_bytes = int(lib().ktau_rank_workspace_size(m, n))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev) if ws_bytes else None
    _check(lib().ktau_rank(_ptr(X), m, n, _ptr(perm), _ptr(rank), _ptr(rstart), _ptr(n1),
                           _ptr(status), _ptr(ws) if ws is not None else None, ws_bytes,
                           _stream(stream)), "ktau_rank")
    if check:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        st = int(status.item())
        if st != 0:
            raise KtauError(st, "ktau_rank")
    u16 = lambda t: t.to(torch.int32) & 0xFFFF  # noqa: E731
    return {"perm": u16(perm), "rank": u16(rank), "rstart": u16(rstart), "n1": n1}


# -------------------------------------------------------------- all-pairs


def ktau_allpairs_workspace_size(m: int, n: int) -> int:
    return int(lib().ktau_allpairs_workspace_size(m, n))


def alloc_outputs(P: int, m: int, device, tau_a: bool = False, counts: bool = True) -> dict:
    out = {"tau_b": torch.empty(P, dtype=torch.float64, device=device),
           "n1": torch.empty(m, dtype=torch.int64, device=device)}
    if counts:
        for k in ("nc", "nd", "n3"):
            out[k] = torch.empty(P, dtype=torch.int64, device=device)
    if tau_a:
        out["tau_a"] = torch.empty(P, dtype=torch.float64, device=device)
    return out


def _pair_out(out: dict) -> _PairOut:
    return _PairOut(*(ctypes.c_void_p(out[k].data_ptr()) if out.get(k) is not None else None
                      for k in ("nc", "nd", "n3", "tau_b", "tau_a", "n1")))


def alloc_workspace(m: int, n: int, device) -> torch.Tensor:
    size = ktau_allpairs_workspace_size(m, n)
    if size == 0:
        raise KtauError(KTAU_EINVAL if n <= KTAU_MAX_N else KTAU_ERANGE, "workspace size")
    return torch.empty(size, dtype=torch.uint8, device=device)


def ktau_allpairs_ex(X: torch.Tensor, J_begin: int, J_end: int, out: dict, workspace: torch.Tensor,
                     scheme=None, q: int = 0, stream=None) -> None:
    X = _as_matrix(X)
    m, n = X.shape
    _check(lib().ktau_allpairs_ex(_ptr(X), m, n, J_begin, J_end, _pair_out(out), _ptr(workspace),
                                  workspace.numel(), scheme_id(scheme), int(q), _stream(stream)),
           "ktau_allpairs_ex")


def ktau_prepare(X: torch.Tensor, workspace: torch.Tensor, n1_out: torch.Tensor | None = None,
                 stream=None) -> None:
    """Rank pre-pass of X into the workspace (first half of ktau_allpairs)."""
    X = _as_matrix(X)
    m, n = X.shape
    _check(lib().ktau_prepare(_ptr(X), m, n, _ptr(n1_out), _ptr(workspace), workspace.numel(),
                              _stream(stream)), "ktau_prepare")


def ktau_pairs(m: int, n: int, out: dict, workspace: torch.Tensor, J_begin: int = -1,
               J_end: int = -1, scheme=None, q: int = 0, stream=None) -> None:
    """Pair kernel over jobs [J_begin, J_end) (all if J_begin < 0) of a
    workspace prepared by ktau_prepare (second half of ktau_allpairs)."""
    _check(lib().ktau_pairs(m, n, J_begin, J_end, _pair_out(out), _ptr(workspace),
                            workspace.numel(), scheme_id(scheme), int(q), _stream(stream)),
           "ktau_pairs")


def ktau_status(workspace: torch.Tensor, stream=None) -> int:
    return int(lib().ktau_status(_ptr(workspace), _stream(stream)))


def ktau_allpairs(X: torch.Tensor, out: dict | None = None, workspace: torch.Tensor | None = None,
                  scheme=None, q: int = 0, tau_a: bool = False, stream=None,
                  check: bool = True) -> dict:
    """All strict pairs of the rows of X (a CUDA float32 m x n tensor).

    Returns a dict of device tensors: nc, nd, n3 (int64), tau_b (and tau_a)
    (float64) indexed by strict job id, and n1 (int64, per row).  With
    check=True the stream is synchronised and a device-side error (NaN input)
    raises KtauError."""
    X = _as_matrix(X)
    m, n = X.shape
    P = m * (m - 1) // 2
    if out is None:
        out = alloc_outputs(P, m, X.device, tau_a=tau_a)
    if workspace is None:
        workspace = alloc_workspace(m, n, X.device)
    if scheme is None and q == 0:
        _check(lib().ktau_allpairs(_ptr(X), m, n, _pair_out(out), _ptr(workspace),
                                   workspace.numel(), _stream(stream)), "ktau_allpairs")
    else:
        ktau_allpairs_ex(X, -1, -1, out, workspace, scheme, q, stream)
    if check:
        st = ktau_status(workspace, stream)
        if st != KTAU_OK:
            raise KtauError(st, "ktau_allpairs")
    return out


def ktau_allpairs_noalloc(X: torch.Tensor, out: dict, status: torch.Tensor | None = None,
                          stream=None) -> None:
    """ktau_allpairs_noalloc: all strict pairs into the caller's output
    tensors with the library's static scratch (no allocation in the call;
    out as from alloc_outputs).  status (a CUDA int32 tensor of one element)
    receives the latched status in stream order."""
    X = _as_matrix(X)
    m, n = X.shape
    _check(lib().ktau_allpairs_noalloc(_ptr(X), m, n, _pair_out(out),
                                       _ptr(status) if status is not None else None,
                                       _stream(stream)), "ktau_allpairs_noalloc")


def ktau_perm_test(X: torch.Tensor, perms: torch.Tensor, J_begin: int = -1, J_end: int = -1,
                   stream=None, check: bool = True) -> dict:
    """Permutation test of every strict pair (or jobs [J_begin, J_end)):
    perms is a CUDA uint16/int16 tensor B x n, each row a permutation of the
    samples applied to the pair's second row.  Returns device tensors
    count (int64: permutations with |n_c - n_d| at least the observed) and
    p (float64: (1 + count) / (B + 1)), indexed by job id - J_begin."""
    X = _as_matrix(X)
    m, n = X.shape
    if perms.dim() != 2 or perms.shape[1] != n or not perms.is_contiguous() or \
            perms.element_size() != 2 or perms.device != X.device:
        raise KtauError(KTAU_EINVAL, "ktau_perm_test: perms must be a contiguous B x n "
                                     "16-bit tensor on the device of X")
    B = perms.shape[0]
    P = m * (m - 1) // 2
    if J_begin < 0:
        J_begin, J_end = 0, P
    size = int(lib().ktau_perm_workspace_size(m, n, B))
    if size == 0:
        raise KtauError(KTAU_EINVAL if n <= KTAU_MAX_N else KTAU_ERANGE, "perm workspace size")
    ws = torch.empty(size, dtype=torch.uint8, device=X.device)
    count = torch.empty(J_end - J_begin, dtype=torch.int64, device=X.device)
    p = torch.empty(J_end - J_begin, dtype=torch.float64, device=X.device)
    _check(lib().ktau_perm_test(_ptr(X), m, n, _ptr(perms), B, J_begin, J_end, _ptr(count),
                                _ptr(p), _ptr(ws), size, _stream(stream)), "ktau_perm_test")
    if check:
        st = ktau_status(ws, stream)
        if st != KTAU_OK:
            raise KtauError(st, "ktau_perm_test")
    return {"count": count, "p": p}


def ktau_allpairs_range(X: torch.Tensor, J_begin: int, J_end: int, out: dict | None = None,
                        workspace: torch.Tensor | None = None, scheme=None, stream=None,
                        check: bool = True) -> dict:
    X = _as_matrix(X)
    m, n = X.shape
    cnt = max(0, J_end - J_begin)
    if out is None:
        out = alloc_outputs(cnt, m, X.device)
    if workspace is None:
        workspace = alloc_workspace(m, n, X.device)
    if scheme is None:
        _check(lib().ktau_allpairs_range(_ptr(X), m, n, J_begin, J_end, _pair_out(out),
                                         _ptr(workspace), workspace.numel(), _stream(stream)),
               "ktau_allpairs_range")
    else:
        ktau_allpairs_ex(X, J_begin, J_end, out, workspace, scheme, 0, stream)
    if check:
        st = ktau_status(workspace, stream)
        if st != KTAU_OK:
            raise KtauError(st, "ktau_allpairs_range")
    return out


# ------------------------------------------------------------------ batched


class _Matrix(ctypes.Structure):
    _fields_ = [("X_dev", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("out", _PairOut)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("force_scheme", ctypes.c_int32), ("force_q", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


def _declare_batch(L):
    i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    decl = {
        "ktau_batch_default_opts": ([p], None),
        "ktau_batch_create": ([p, i64, p, p, p], i32),
        "ktau_batch_run": ([p, p], i32),
        "ktau_batch_status": ([p, p], i32),
        "ktau_batch_plan": ([p, i64, p, p], i32),
        "ktau_batch_destroy": ([p], None),
        "ktau_autotune": ([p, i64, ctypes.c_char_p, p, p, p], i32),
    }
    for name, (args, res) in decl.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def _blib():
    L = lib()
    if not hasattr(L, "_ktau_batch_declared"):
        _declare_batch(L)
        L._ktau_batch_declared = True
    return L


class KtauBatch:
    """A batch plan (ktau_batch_create) over CUDA float32 matrices.

    ``outs[i]`` is a dict of result tensors like alloc_outputs() returns; if
    omitted they are allocated.  The tensors are kept alive by the plan."""

    def __init__(self, mats, outs=None, use_graph=True, autotune=True, force_scheme=None,
                 force_q=0, tune_cache=None, stream=None):
        L = _blib()
        self._mats = [_as_matrix(X) for X in mats]
        if outs is None:
            outs = [alloc_outputs(X.shape[0] * (X.shape[0] - 1) // 2, X.shape[0], X.device)
                    for X in self._mats]
        self.outs = outs
        arr = (_Matrix * len(self._mats))()
        for i, (X, o) in enumerate(zip(self._mats, outs)):
            arr[i] = _Matrix(ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1], _pair_out(o))
        opts = _BatchOpts()
        L.ktau_batch_default_opts(ctypes.byref(opts))
        opts.use_graph = 1 if use_graph else 0
        opts.autotune = 1 if autotune else 0
        opts.force_scheme = -1 if force_scheme is None else scheme_id(force_scheme)
        opts.force_q = int(force_q)
        self._cache = tune_cache.encode() if tune_cache else None
        opts.tune_cache = self._cache
        h = ctypes.c_void_p()
        _check(L.ktau_batch_create(arr, len(self._mats), ctypes.byref(opts), _stream(stream),
                                   ctypes.byref(h)), "ktau_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(_blib().ktau_batch_run(self._h, _stream(stream)), "ktau_batch_run")

    def status(self, stream=None) -> int:
        return int(_blib().ktau_batch_status(self._h, _stream(stream)))

    def plan(self, i: int) -> tuple[str, int]:
        s, q = ctypes.c_int32(), ctypes.c_int32()
        _check(_blib().ktau_batch_plan(self._h, i, ctypes.byref(s), ctypes.byref(q)),
               "ktau_batch_plan")
        return scheme_name(s.value), q.value

    def close(self):
        if getattr(self, "_h", None):
            _blib().ktau_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ktau_autotune(ns, cache_path: str | None = None, stream=None) -> list[tuple[str, int]]:
    L = _blib()
    arr = (ctypes.c_int64 * len(ns))(*ns)
    sch = (ctypes.c_int32 * len(ns))()
    qs = (ctypes.c_int32 * len(ns))()
    _check(L.ktau_autotune(arr, len(ns), cache_path.encode() if cache_path else None,
                           _stream(stream), sch, qs), "ktau_autotune")
    return [(scheme_name(s), q) for s, q in zip(sch, qs)]


# ------------------------------------------------------------ diagnostics


def probe_peaks(blocks: int = 2048, valu_iters: int = 20000, lds_iters: int = 2000,
                stream=None) -> dict:
    """Measured int32 VALU lane-operations/s and LDS bytes/s from the
    library's probe kernels (each timed with events on `stream`, best of
    three launches after a warm-up)."""
    L = lib()
    threads = L.ktau_probe_threads()
    out = torch.empty(blocks * threads, dtype=torch.int32, device="cuda")
    st = stream or torch.cuda.current_stream()

    def best(fn, iters):
        _check(fn(_ptr(out), blocks, iters, _stream(st)), "probe")
        ms = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            _check(fn(_ptr(out), blocks, iters, _stream(st)), "probe")
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms)

    v_ms = best(L.ktau_probe_valu, valu_iters)
    l_ms = best(L.ktau_probe_lds, lds_iters)
    ops = blocks * threads * L.ktau_probe_valu_ops_per_iter() * valu_iters
    byt = blocks * threads * L.ktau_probe_lds_bytes_per_iter() * lds_iters
    # wave instructions per second of each instruction kind of the issue probe
    issue = {}
    for kind, name in enumerate(ISSUE_KINDS):
        ms = best(lambda o, b, i, s, kind=kind: L.ktau_probe_issue(o, b, i, kind, s), valu_iters)
        waves = blocks * threads // 64
        issue[name] = waves * L.ktau_probe_issue_instrs_per_iter(kind) * valu_iters / (ms * 1e-3)
    return {"valu_lane_ops_per_s": ops / (v_ms * 1e-3), "lds_bytes_per_s": byt / (l_ms * 1e-3),
            "valu_ms": v_ms, "lds_ms": l_ms, "issue_wave_instr_per_s": issue}


# Instruction kinds of the issue-rate probe, in the library's order.
ISSUE_KINDS = ("v_add_u32", "v_pk_minimum3_f16", "v_dot2_u32_u16", "v_pk_min_u16+v_pk_add_u16")

