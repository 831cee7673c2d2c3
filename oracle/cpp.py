"""The C++/OpenMP form of the FP64 oracle (``katz_ref.cpp``), for graphs too
large for the numpy oracle (R-MAT scale 27: 4.3e9 arcs) and for the CPU
baseline on all host cores.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It computes what
``oracle.katz.rank_static`` / ``oracle.katz.bounds`` compute, bit for bit, for
any thread count; the tests pin it against that oracle and through the same
closed forms and exact rankings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .katz import OracleResult

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "katz_ref.cpp")
LIB_PATH = os.path.join(_HERE, "libkatz_ref.so")
_lib = None

# -O3 without -march: the library is compiled here and may run on a host with
# another CPU; the walk is bound by memory gathers, not by vector width.
FLAGS = ["-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile ``katz_ref.cpp`` into ``libkatz_ref.so`` with g++."""
    global _lib
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["g++", *FLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, LIB_PATH)
        _lib = None
    return LIB_PATH


class _Res(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("rest_upper_max", ctypes.c_double), ("active_final", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("status", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run oracle.cpp.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.ko_rank_static.restype = ctypes.c_int
        lib.ko_rank_static.argtypes = [i64, vp, vp, f64, i64, f64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                       ctypes.POINTER(_Res)]
        lib.ko_bounds.restype = ctypes.c_int
        lib.ko_bounds.argtypes = [i64, vp, vp, f64, i32, i32, i32, vp, vp]
        lib.ko_walk_rows.restype = ctypes.c_int
        lib.ko_walk_rows.argtypes = [i64, vp, vp, f64, i64, i64, i32, vp, vp]
        lib.ko_max_threads.restype = ctypes.c_int
        lib.ko_max_threads.argtypes = []
        _lib = lib
    return _lib


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return rp, cl


def max_threads() -> int:
    return int(_load().ko_max_threads())


def rank_static(row_ptr, col, alpha=None, k=10, eps=0.0, undirected=True, max_iter=1000, threads=0,
                full=True):
    """Algorithm 1 with the top-k criterion (same arguments and result as
    ``oracle.katz.rank_static``).  ``full=False`` skips the per-node arrays
    (c, x, lower_all, upper_all are then None) to save host memory on large
    graphs; ``threads`` = 0 uses every OpenMP thread."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    topk = np.empty(k, dtype=np.int32)
    lo = np.empty(k, dtype=np.float64)
    up = np.empty(k, dtype=np.float64)
    arrays = [np.empty(n, dtype=np.float64) for _ in range(4)] if full else [None] * 4
    res = _Res()
    ptr = [a.ctypes.data if a is not None else None for a in arrays]
    rc = _load().ko_rank_static(n, rp.ctypes.data, cl.ctypes.data, 0.0 if alpha is None else float(alpha),
                                int(k), float(eps), int(bool(undirected)), int(max_iter), int(threads),
                                topk.ctypes.data, lo.ctypes.data, up.ctypes.data, *ptr, ctypes.byref(res))
    if rc == -1:
        raise ValueError("invalid arguments (alpha, k, eps or max_iter)")
    if rc != 0:
        raise MemoryError("C++ oracle ran out of host memory")
    c, x, lo_all, up_all = arrays
    return OracleResult(topk=topk.astype(np.int64), lower=lo, upper=up, iterations=res.iterations,
                        status=res.status, rest_upper_max=res.rest_upper_max, active_final=res.active_final,
                        alpha=res.alpha, gamma=res.gamma, beta=res.beta, c=c, x=x, lower_all=lo_all,
                        upper_all=up_all, active=None)


def bounds(row_ptr, col, alpha=None, r=1, undirected=True, threads=0):
    """l_r and u_r of every node after exactly r iterations (``oracle.katz.bounds``)."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    lo = np.empty(n, dtype=np.float64)
    up = np.empty(n, dtype=np.float64)
    rc = _load().ko_bounds(n, rp.ctypes.data, cl.ctypes.data, 0.0 if alpha is None else float(alpha), int(r),
                           int(bool(undirected)), int(threads), lo.ctypes.data, up.ctypes.data)
    if rc == -1:
        raise ValueError("invalid arguments (alpha or r)")
    if rc != 0:
        raise MemoryError("C++ oracle ran out of host memory")
    return lo, up


def walk_rows(row_ptr, col, alpha, lo, hi, x_in, threads=0):
    """One walk step, x_out = alpha (A x_in) on rows lo..hi-1 (the iteration's
    own loop), for timing a bounded sample of a large graph."""
    rp, cl = _csr(row_ptr, col)
    x = np.ascontiguousarray(x_in, dtype=np.float64)
    out = np.empty(max(hi - lo, 1), dtype=np.float64)
    rc = _load().ko_walk_rows(rp.size - 1, rp.ctypes.data, cl.ctypes.data, float(alpha), int(lo), int(hi),
                              int(threads), x.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid row range")
    return out[:hi - lo]
