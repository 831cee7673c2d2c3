"""Thin Python binding of ``libkatz.so`` (the C ABI in ``include/katz.h``).

Argument marshalling only: every step of the ranking runs in the HIP library.
Torch tensors provide device memory and streams.  Importing this module fails
loudly when the compiled library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkatz.so")

OK = 0
W_ITER_LIMIT = 1
W_PRECISION_LIMIT = 2
W_EXACT_TIES = 3
E_INVALID_ARG = -1
E_ALPHA = -2
E_CSR = -3
E_UPDATE = -4
E_DEGREE_CAP = -5
E_OOM = -6
E_HIP = -7
E_UNSUPPORTED = -8
E_SCRATCH = -9
E_CANCELLED = -10
E_TIMEOUT = -11
E_BUSY = -12

FP64 = 0
FP32_MARGIN = 1
TOPK, RANKING, SCORE, PAIR = 0, 1, 2, 3
CRITERIA = {"topk": TOPK, "ranking": RANKING, "score": SCORE, "pair": PAIR}
VALIDATE_NONE, VALIDATE_BASIC, VALIDATE_STRICT = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32_MARGIN}


class KatzCSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("row_ptr_64", ctypes.c_int32), ("undirected", ctypes.c_int32)]


class KatzParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("epsilon", ctypes.c_double), ("k", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32), ("criterion", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("flags", ctypes.c_int32), ("degree_cap", ctypes.c_int64),
                ("pair_u", ctypes.c_int32), ("pair_v", ctypes.c_int32)]


class KatzResult(ctypes.Structure):
    _fields_ = [("topk_ids", ctypes.c_void_p), ("lower", ctypes.c_void_p), ("upper", ctypes.c_void_p),
                ("rest_upper_max", ctypes.c_double), ("alpha_used", ctypes.c_double),
                ("eta", ctypes.c_double), ("active_final", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("separated_fraction", ctypes.c_double)]


class KatzSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("residual", ctypes.c_double),
                ("alpha_used", ctypes.c_double)]


SOLVE_FOSTER, SOLVE_CG = 0, 1
SOLVE_METHODS = {"foster": SOLVE_FOSTER, "cg": SOLVE_CG}


class KatzTuning(ctypes.Structure):
    _fields_ = [("hub_bytes", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("batch_blocks_per_cu", ctypes.c_int32), ("batch_tile", ctypes.c_int32),
                ("batch_xcd", ctypes.c_int32), ("walk_groups", ctypes.c_int32), ("split_hot_bytes", ctypes.c_int32),
                ("bin_bounds", ctypes.c_int32 * 6), ("reserved", ctypes.c_int32)]


class KatzTiming(ctypes.Structure):
    _fields_ = [("walk_step_ms", ctypes.c_double), ("walk_step_launches", ctypes.c_int64),
                ("walk_first_ms", ctypes.c_double), ("walk_first_launches", ctypes.c_int64),
                ("select_ms", ctypes.c_double), ("select_iterations", ctypes.c_int64),
                ("prep_ms", ctypes.c_double), ("result_ms", ctypes.c_double),
                ("call_ms", ctypes.c_double), ("calls", ctypes.c_int64),
                ("renumber_step_ms", ctypes.c_double), ("renumber_step_launches", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1807_03847_amd._build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.katz_autotune_cache.restype = ctypes.c_int
    lib.katz_autotune_cache.argtypes = [ctypes.c_char_p]
    lib.katz_rank_static.restype = ctypes.c_int
    lib.katz_rank_static.argtypes = [i32, ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams),
                                     ctypes.POINTER(KatzResult), ctypes.POINTER(vp), vp]
    lib.katz_rank_static_noalloc.restype = ctypes.c_int
    lib.katz_rank_static_noalloc.argtypes = [ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams),
                                             ctypes.POINTER(KatzResult), vp]
    lib.katz_solve.restype = ctypes.c_int
    lib.katz_solve.argtypes = [ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams), i32, ctypes.c_double, vp,
                               ctypes.POINTER(KatzSolveInfo), vp]
    lib.katz_rank_update.restype = ctypes.c_int
    lib.katz_rank_update.argtypes = [vp, vp, vp, i64, vp, vp, i64, ctypes.POINTER(KatzResult), vp]
    lib.katz_bounds.restype = ctypes.c_int
    lib.katz_bounds.argtypes = [ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams), i32, vp, vp, vp]
    lib.katz_state_free.restype = None
    lib.katz_state_free.argtypes = [vp]
    lib.katz_strerror.restype = ctypes.c_char_p
    lib.katz_strerror.argtypes = [ctypes.c_int]
    lib.katz_server_create.restype = ctypes.c_int
    lib.katz_server_create.argtypes = [i32, i64, ctypes.POINTER(vp)]
    lib.katz_server_add_graph.restype = ctypes.c_int
    lib.katz_server_add_graph.argtypes = [vp, ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams),
                                          ctypes.POINTER(KatzResult), ctypes.POINTER(i32)]
    lib.katz_server_submit.restype = ctypes.c_int
    lib.katz_server_submit.argtypes = [vp, i32, vp, vp, i64, vp, vp, i64, ctypes.POINTER(i64)]
    lib.katz_server_wait.restype = ctypes.c_int
    lib.katz_server_wait.argtypes = [vp, i64, ctypes.POINTER(KatzResult), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.katz_server_wait_for.restype = ctypes.c_int
    lib.katz_server_wait_for.argtypes = [vp, i64, i64, ctypes.POINTER(KatzResult), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    lib.katz_server_cancel.restype = ctypes.c_int
    lib.katz_server_cancel.argtypes = [vp, i64]
    lib.katz_state_save.restype = ctypes.c_int
    lib.katz_state_save.argtypes = [vp, ctypes.c_char_p]
    lib.katz_state_load.restype = ctypes.c_int
    lib.katz_state_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp), vp]
    lib.katz_state_size.restype = ctypes.c_int
    lib.katz_state_size.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.katz_server_destroy.restype = None
    lib.katz_server_destroy.argtypes = [vp]
    lib.katz_timing_enable.restype = None
    lib.katz_timing_enable.argtypes = [ctypes.c_int]
    lib.katz_timing_read.restype = ctypes.c_int
    lib.katz_timing_read.argtypes = [ctypes.POINTER(KatzTiming)]
    lib.katz_tuning_get.restype = ctypes.c_int
    lib.katz_tuning_get.argtypes = [ctypes.POINTER(KatzTuning)]
    lib.katz_tuning_set.restype = ctypes.c_int
    lib.katz_tuning_set.argtypes = [ctypes.POINTER(KatzTuning)]
    lib.katz_autotune.restype = ctypes.c_int
    lib.katz_autotune.argtypes = [i32, ctypes.POINTER(KatzCSR), ctypes.POINTER(KatzParams), ctypes.POINTER(KatzTuning),
                                  vp]
    return lib


lib = _load()


class KatzError(RuntimeError):
    def __init__(self, code: int):
        self.code = code
        super().__init__(f"katz error {code}: {strerror(code)}")


def strerror(code: int) -> str:
    return lib.katz_strerror(code).decode()


@dataclass
class RankResult:
    topk: torch.Tensor          # int32 [k] node ids in ranking order
    lower: torch.Tensor         # float64 [k]
    upper: torch.Tensor         # float64 [k]
    iterations: int
    status: int
    rest_upper_max: float
    alpha: float
    eta: float
    active_final: int
    separated_fraction: float = math.nan   # ranking and score criteria only


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream, device):
    if device.type != "cuda":
        return ctypes.c_void_p(0)
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def make_csr(row_ptr: torch.Tensor, col: torch.Tensor, undirected: bool = True) -> KatzCSR:
    if row_ptr.dtype not in (torch.int32, torch.int64) or col.dtype != torch.int32:
        raise TypeError("row_ptr must be int32/int64 and col int32")
    if not (row_ptr.is_contiguous() and col.is_contiguous()):
        raise ValueError("row_ptr and col must be contiguous")
    n = row_ptr.numel() - 1
    return KatzCSR(n=n, nnz=col.numel(), row_ptr=row_ptr.data_ptr(), col=col.data_ptr() if col.numel() else 0,
                   row_ptr_64=int(row_ptr.dtype == torch.int64), undirected=int(bool(undirected)))


FLAG_NO_REORDER = 1
FLAG_REORDER = 2
FLAG_INBOUND = 4


def make_params(k=1, alpha=0.0, eps=0.0, precision="fp64", max_iter=0, validate=VALIDATE_BASIC,
                degree_cap=0, flags=0, criterion="topk", pair=(0, 0)) -> KatzParams:
    return KatzParams(alpha=float(alpha), epsilon=float(eps), k=int(k), max_iter=int(max_iter),
                      precision=PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                      criterion=CRITERIA[criterion] if isinstance(criterion, str) else int(criterion),
                      validate=int(validate), flags=int(flags), degree_cap=int(degree_cap),
                      pair_u=int(pair[0]), pair_v=int(pair[1]))


def _alloc_outputs(k, device):
    return (torch.empty(k, dtype=torch.int32, device=device),
            torch.empty(k, dtype=torch.float64, device=device),
            torch.empty(k, dtype=torch.float64, device=device))


def _to_result(res: KatzResult, ids, lo, up) -> RankResult:
    return RankResult(topk=ids, lower=lo, upper=up, iterations=res.iterations, status=res.status,
                      rest_upper_max=res.rest_upper_max, alpha=res.alpha_used, eta=res.eta,
                      active_final=res.active_final, separated_fraction=res.separated_fraction)


def rank_static(row_ptr, col, k, *, alpha=0.0, eps=0.0, precision="fp64", undirected=True, max_iter=0,
                validate=VALIDATE_BASIC, flags=0, stream=None, out=None, criterion="topk",
                pair=(0, 0)) -> RankResult:
    """katz_rank_static for one graph (Algorithm 1) with a stopping criterion
    of Section 3.1: "topk" (k nodes), "ranking" and "score" (every node; k is
    ignored) or "pair" (the two nodes of ``pair``; k is ignored).

    ``out`` may pass preallocated (ids, lower, upper) tensors of the output length."""
    device = row_ptr.device
    g = make_csr(row_ptr, col, undirected)
    p = make_params(k, alpha, eps, precision, max_iter, validate, 0, flags, criterion, pair)
    length = {TOPK: p.k, RANKING: g.n, SCORE: g.n, PAIR: 2}.get(p.criterion, p.k)
    ids, lo, up = out if out is not None else _alloc_outputs(max(length, 0), device)
    res = KatzResult(topk_ids=ids.data_ptr(), lower=lo.data_ptr(), upper=up.data_ptr())
    rc = lib.katz_rank_static(1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(res), None,
                              _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return _to_result(res, ids, lo, up)


def rank_static_noalloc(row_ptr, col, k, *, alpha=0.0, eps=0.0, precision="fp64", undirected=True, max_iter=0,
                        validate=VALIDATE_BASIC, flags=0, stream=None, out=None, criterion="topk",
                        pair=(0, 0)) -> RankResult:
    """katz_rank_static_noalloc: rank_static in the library's fixed scratch
    array, without any allocation by the library.  Pass ``out`` to avoid the
    output allocation here as well."""
    device = row_ptr.device
    g = make_csr(row_ptr, col, undirected)
    p = make_params(k, alpha, eps, precision, max_iter, validate, 0, flags, criterion, pair)
    length = {TOPK: p.k, RANKING: g.n, SCORE: g.n, PAIR: 2}.get(p.criterion, p.k)
    ids, lo, up = out if out is not None else _alloc_outputs(max(length, 0), device)
    res = KatzResult(topk_ids=ids.data_ptr(), lower=lo.data_ptr(), upper=up.data_ptr())
    rc = lib.katz_rank_static_noalloc(ctypes.byref(g), ctypes.byref(p), ctypes.byref(res),
                                      _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return _to_result(res, ids, lo, up)


def solve(row_ptr, col, method="cg", tol=1e-15, *, alpha=0.0, max_iter=0, undirected=True,
          validate=VALIDATE_BASIC, flags=0, stream=None, out=None):
    """katz_solve: Katz scores of every node by Foster's heuristic ("foster")
    or by conjugate gradients on Eq. (la) ("cg").  Returns (scores, info dict,
    status)."""
    device = row_ptr.device
    g = make_csr(row_ptr, col, undirected)
    p = make_params(1, alpha, 0.0, "fp64", max_iter, validate, 0, flags)
    scores = out if out is not None else torch.empty(g.n, dtype=torch.float64, device=device)
    info = KatzSolveInfo()
    rc = lib.katz_solve(ctypes.byref(g), ctypes.byref(p), SOLVE_METHODS[method] if isinstance(method, str)
                        else int(method), float(tol), _ptr(scores), ctypes.byref(info),
                        _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return scores, {name: getattr(info, name) for name, _ in KatzSolveInfo._fields_}, rc


def rank_static_batch(graphs, params, *, stream=None):
    """katz_rank_static with count = len(graphs).

    graphs: list of (row_ptr, col, undirected); params: list of dicts with the
    keyword arguments of ``make_params``."""
    count = len(graphs)
    device = graphs[0][0].device
    G = (KatzCSR * count)(*[make_csr(rp, c, u) for rp, c, u in graphs])
    P = (KatzParams * count)(*[make_params(**pp) for pp in params])
    outs = [_alloc_outputs(pp["k"], device) for pp in params]
    R = (KatzResult * count)(*[KatzResult(topk_ids=i.data_ptr(), lower=l.data_ptr(), upper=u.data_ptr())
                               for i, l, u in outs])
    rc = lib.katz_rank_static(count, G, P, R, None, _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return [_to_result(R[i], *outs[i]) for i in range(count)]


def bounds(row_ptr, col, r, *, alpha=0.0, precision="fp64", undirected=True, validate=VALIDATE_BASIC,
           flags=0, stream=None):
    """katz_bounds: (lower, upper) of every node after exactly r iterations."""
    device = row_ptr.device
    g = make_csr(row_ptr, col, undirected)
    p = make_params(1, alpha, 0.0, precision, 0, validate, 0, flags)
    n = row_ptr.numel() - 1
    lo = torch.empty(n, dtype=torch.float64, device=device)
    up = torch.empty(n, dtype=torch.float64, device=device)
    rc = lib.katz_bounds(ctypes.byref(g), ctypes.byref(p), int(r), _ptr(lo), _ptr(up),
                         _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return lo, up


class State:
    """A dynamic ranking state (katz_state): the graph, the walk history, c_r and
    M on the device.  ``update`` applies one batch of edge (undirected graph) or
    arc (directed graph) insertions and deletions (Algorithm 2) and returns the
    re-certified top-k."""

    def __init__(self, handle, k, device):
        self._h = handle
        self.k = k
        self.device = device

    def update(self, ins=None, dels=None, *, stream=None, out=None) -> RankResult:
        import numpy as np
        ins = np.asarray(ins if ins is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        dels = np.asarray(dels if dels is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        iu, iv = np.ascontiguousarray(ins[:, 0]), np.ascontiguousarray(ins[:, 1])
        du, dv = np.ascontiguousarray(dels[:, 0]), np.ascontiguousarray(dels[:, 1])
        ids, lo, up = out if out is not None else _alloc_outputs(self.k, self.device)
        res = KatzResult(topk_ids=ids.data_ptr(), lower=lo.data_ptr(), upper=up.data_ptr())
        rc = lib.katz_rank_update(ctypes.c_void_p(self._h), iu.ctypes.data, iv.ctypes.data, len(iu),
                                  du.ctypes.data, dv.ctypes.data, len(du), ctypes.byref(res),
                                  _stream_handle(stream, self.device))
        if rc < 0:
            raise KatzError(rc)
        return _to_result(res, ids, lo, up)

    def save(self, path) -> None:
        """katz_state_save: writes the state to a file (a checkpoint)."""
        rc = lib.katz_state_save(ctypes.c_void_p(self._h), os.fsencode(path))
        if rc < 0:
            raise KatzError(rc)

    def free(self):
        if self._h:
            lib.katz_state_free(ctypes.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def create_state(row_ptr, col, k, *, alpha=0.0, eps=0.0, max_iter=0, degree_cap=0, validate=VALIDATE_BASIC,
                 flags=0, undirected=True, precision="fp64", stream=None):
    """katz_rank_static with a state: ranks the graph (Algorithm 1, FP64 or
    FP32 form, kept walk history) and returns (State, RankResult) for later
    updates.  A directed graph's update pairs (u, v) are arcs u -> v; with
    FLAG_INBOUND the state ranks by inbound walks."""
    device = row_ptr.device
    g = make_csr(row_ptr, col, undirected)
    p = make_params(k, alpha, eps, precision, max_iter, validate, degree_cap, flags)
    ids, lo, up = _alloc_outputs(k, device)
    res = KatzResult(topk_ids=ids.data_ptr(), lower=lo.data_ptr(), upper=up.data_ptr())
    handle = ctypes.c_void_p(0)
    rc = lib.katz_rank_static(1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(res), ctypes.byref(handle),
                              _stream_handle(stream, device))
    if rc < 0:
        raise KatzError(rc)
    return State(handle.value, k, device), _to_result(res, ids, lo, up)


def load_state(path, device=None, stream=None) -> State:
    """katz_state_load: a state restored from a checkpoint file on the current
    (or given) device."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = ctypes.c_void_p(0)
    rc = lib.katz_state_load(os.fsencode(path), ctypes.byref(h), _stream_handle(stream, dev))
    if rc < 0:
        raise KatzError(rc)
    k = ctypes.c_int32(0)
    lib.katz_state_size(h, None, ctypes.byref(k))
    return State(h.value, k.value, dev)


class Server:
    """katz_server: worker slots with their own streams, per-graph FIFO order,
    admission by free slots and a device-memory budget."""

    def __init__(self, slots=4, memory_budget=0):
        h = ctypes.c_void_p(0)
        rc = lib.katz_server_create(int(slots), int(memory_budget), ctypes.byref(h))
        if rc < 0:
            raise KatzError(rc)
        self._h = h.value
        self._k = {}

    def add_graph(self, row_ptr, col, k, *, alpha=0.0, eps=0.0, max_iter=0, degree_cap=0,
                  validate=VALIDATE_BASIC, flags=0, undirected=True, precision="fp64"):
        """Registers a graph (host or device CSR); returns (graph_id, initial RankResult on the host)."""
        import numpy as np
        g = make_csr(row_ptr, col, undirected)
        p = make_params(k, alpha, eps, precision, max_iter, validate, degree_cap, flags)
        ids = np.empty(k, dtype=np.int32)
        lo = np.empty(k, dtype=np.float64)
        up = np.empty(k, dtype=np.float64)
        res = KatzResult(topk_ids=ids.ctypes.data, lower=lo.ctypes.data, upper=up.ctypes.data)
        gid = ctypes.c_int32(0)
        rc = lib.katz_server_add_graph(ctypes.c_void_p(self._h), ctypes.byref(g), ctypes.byref(p),
                                       ctypes.byref(res), ctypes.byref(gid))
        if rc < 0:
            raise KatzError(rc)
        self._k[gid.value] = k
        return gid.value, _to_result(res, ids, lo, up)

    def submit(self, graph_id, ins=None, dels=None) -> int:
        import numpy as np
        ins = np.asarray(ins if ins is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        dels = np.asarray(dels if dels is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        iu, iv = np.ascontiguousarray(ins[:, 0]), np.ascontiguousarray(ins[:, 1])
        du, dv = np.ascontiguousarray(dels[:, 0]), np.ascontiguousarray(dels[:, 1])
        t = ctypes.c_int64(0)
        rc = lib.katz_server_submit(ctypes.c_void_p(self._h), int(graph_id), iu.ctypes.data, iv.ctypes.data,
                                    len(iu), du.ctypes.data, dv.ctypes.data, len(du), ctypes.byref(t))
        if rc < 0:
            raise KatzError(rc)
        self._k[("t", t.value)] = self._k[graph_id]
        return t.value

    def wait(self, ticket, timeout_ms=None):
        """Returns (RankResult with host arrays, latency_ms, service_ms); raises on
        errors.  With timeout_ms, katz_server_wait_for: KatzError(E_TIMEOUT)
        leaves the ticket valid."""
        import numpy as np
        k = self._k[("t", ticket)]
        ids = np.empty(k, dtype=np.int32)
        lo = np.empty(k, dtype=np.float64)
        up = np.empty(k, dtype=np.float64)
        res = KatzResult(topk_ids=ids.ctypes.data, lower=lo.ctypes.data, upper=up.ctypes.data)
        lat = ctypes.c_double(0)
        svc = ctypes.c_double(0)
        if timeout_ms is None:
            rc = lib.katz_server_wait(ctypes.c_void_p(self._h), int(ticket), ctypes.byref(res), ctypes.byref(lat),
                                      ctypes.byref(svc))
        else:
            rc = lib.katz_server_wait_for(ctypes.c_void_p(self._h), int(ticket), int(timeout_ms), ctypes.byref(res),
                                          ctypes.byref(lat), ctypes.byref(svc))
        if rc != E_TIMEOUT:
            self._k.pop(("t", ticket), None)
        if rc < 0:
            raise KatzError(rc)
        return _to_result(res, ids, lo, up), lat.value, svc.value

    def cancel(self, ticket) -> int:
        """katz_server_cancel: OK, or raises KatzError(E_BUSY / E_INVALID_ARG)."""
        rc = lib.katz_server_cancel(ctypes.c_void_p(self._h), int(ticket))
        if rc < 0:
            raise KatzError(rc)
        return rc

    def close(self):
        if self._h:
            lib.katz_server_destroy(ctypes.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tuning_dict(t):
    return {"hub_bytes": t.hub_bytes, "blocks_per_cu": t.blocks_per_cu, "batch_blocks_per_cu": t.batch_blocks_per_cu,
            "batch_tile": t.batch_tile, "batch_xcd": t.batch_xcd, "walk_groups": t.walk_groups,
            "split_hot_bytes": t.split_hot_bytes, "bin_bounds": list(t.bin_bounds)}


def tuning_get() -> dict:
    """katz_tuning_get: the walk kernels' launch shape."""
    t = KatzTuning()
    rc = lib.katz_tuning_get(ctypes.byref(t))
    if rc < 0:
        raise KatzError(rc)
    return _tuning_dict(t)


def tuning_set(hub_bytes=0, blocks_per_cu=0, batch_blocks_per_cu=0, batch_tile=0, batch_xcd=0,
               walk_groups=0, split_hot_bytes=0, bin_bounds=None) -> None:
    """katz_tuning_set (no result depends on it, except on split_hot_bytes and
    bin_bounds, which change the order of additions)."""
    bb = [int(v) for v in (bin_bounds if bin_bounds is not None else [0] * 6)]
    t = KatzTuning(hub_bytes=int(hub_bytes), blocks_per_cu=int(blocks_per_cu),
                   batch_blocks_per_cu=int(batch_blocks_per_cu), batch_tile=int(batch_tile),
                   batch_xcd=int(batch_xcd), walk_groups=int(walk_groups), split_hot_bytes=int(split_hot_bytes),
                   bin_bounds=(ctypes.c_int32 * 6)(*bb))
    rc = lib.katz_tuning_set(ctypes.byref(t))
    if rc < 0:
        raise KatzError(rc)


def autotune(row_ptr, col, k, *, alpha=0.0, eps=0.0, precision="fp32", undirected=True, stream=None) -> dict:
    """katz_autotune for one graph: times the candidate launch shapes and keeps the fastest."""
    g = make_csr(row_ptr, col, undirected)
    p = make_params(k, alpha, eps, precision)
    t = KatzTuning()
    rc = lib.katz_autotune(1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(t),
                           _stream_handle(stream, row_ptr.device))
    if rc < 0:
        raise KatzError(rc)
    return _tuning_dict(t)


def autotune_cache(path=None) -> None:
    """katz_autotune_cache: keep autotuner results in a text file (None: off)."""
    lib.katz_autotune_cache(None if path is None else os.fsencode(str(path)))


def autotune_batch(graphs, params, *, stream=None) -> dict:
    """katz_autotune for a batch (same arguments as ``rank_static_batch``)."""
    count = len(graphs)
    G = (KatzCSR * count)(*[make_csr(rp, c, u) for rp, c, u in graphs])
    P = (KatzParams * count)(*[make_params(**pp) for pp in params])
    t = KatzTuning()
    rc = lib.katz_autotune(count, G, P, ctypes.byref(t), _stream_handle(stream, graphs[0][0].device))
    if rc < 0:
        raise KatzError(rc)
    return _tuning_dict(t)


def timing_enable(on: bool = True) -> None:
    """Reset the library's device-time counters and start (or stop) recording."""
    lib.katz_timing_enable(int(bool(on)))


def timing_read() -> dict:
    t = KatzTiming()
    lib.katz_timing_read(ctypes.byref(t))
    return {name: getattr(t, name) for name, _ in KatzTiming._fields_}


NEG_INF = -math.inf
