"""Seeded synthetic graphs in CSR form (input data for the library, its tests and
its benchmark).

This module generates inputs only; it holds none of the Katz method's arithmetic.
Large generators (Erdos-Renyi, R-MAT, Barabasi-Albert) run in ``gen.cpp`` through
ctypes; the small fixed shapes used by the tests (complete graph, cycle, star,
path, random small graphs) are written here in numpy.

Every graph is returned as ``(row_ptr, col)``: ``row_ptr`` int64 of length n + 1,
``col`` int32 of length nnz.  Undirected graphs store both arcs of every edge;
rows are sorted, duplicate-free and loop-free.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynthgraph.so")
_GPU_LIB_PATH = os.path.join(_HERE, "libsynthgraph_gpu.so")
_lib = None
_gpu_lib = None
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(force: bool = True) -> str:
    """Compile ``gen.cpp`` into ``libsynthgraph.so`` (g++ with OpenMP) and
    ``gen_gpu.hip`` into ``libsynthgraph_gpu.so`` (hipcc, gfx950)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "gen.cpp"), "-o", _LIB_PATH + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    if force or not os.path.exists(_GPU_LIB_PATH):
        cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(_HERE, "gen_gpu.hip"), "-o", _GPU_LIB_PATH + ".tmp"]
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + proc.stdout + proc.stderr)
        os.replace(_GPU_LIB_PATH + ".tmp", _GPU_LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run synthgraph.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.sg_er.restype = vp
    lib.sg_er.argtypes = [i64, i64, u64]
    lib.sg_rmat.restype = vp
    lib.sg_rmat.argtypes = [i32, i32, f64, f64, f64, u64, i32]
    lib.sg_ba.restype = vp
    lib.sg_ba.argtypes = [i64, i32, u64]
    lib.sg_n.restype = i64
    lib.sg_n.argtypes = [vp]
    lib.sg_nnz.restype = i64
    lib.sg_nnz.argtypes = [vp]
    lib.sg_export.restype = None
    lib.sg_export.argtypes = [vp, vp, vp]
    lib.sg_detach.restype = None
    lib.sg_detach.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.sg_free_array.restype = None
    lib.sg_free_array.argtypes = [vp]
    lib.sg_free.restype = None
    lib.sg_free.argtypes = [vp]
    lib.sg_permutation.restype = None
    lib.sg_permutation.argtypes = [i64, u64, vp]
    lib.sg_rmat_pairs.restype = None
    lib.sg_rmat_pairs.argtypes = [i32, f64, f64, f64, u64, i32, u64, u64, i64, vp, vp]
    lib.sg_draw.restype = None
    lib.sg_draw.argtypes = [u64, u64, u64, i64, vp]
    _lib = lib
    return lib


def _own(ptr, count, ctype, dtype):
    """A numpy array over `count` elements of generator-allocated memory; the
    memory is freed (sg_free_array) when the last view of it is gone."""
    lib = _load()
    if count == 0:
        lib.sg_free_array(ptr)
        return np.empty(0, dtype=dtype)
    buf = (ctype * count).from_address(ptr)
    arr = np.ctypeslib.as_array(buf)
    weakref.finalize(buf, lib.sg_free_array, ptr)
    assert arr.dtype == dtype
    return arr


def _take(handle):
    """The generated CSR, without copying: large graphs (R-MAT scale 27 holds
    4.3e9 arcs) are handed over as they are."""
    lib = _load()
    if not handle:
        raise ValueError("graph generator rejected its arguments or ran out of memory")
    n = lib.sg_n(handle)
    nnz = lib.sg_nnz(handle)
    rp_p = ctypes.c_void_p()
    col_p = ctypes.c_void_p()
    lib.sg_detach(handle, ctypes.byref(rp_p), ctypes.byref(col_p))
    row_ptr = _own(rp_p.value, n + 1, ctypes.c_int64, np.int64)
    col = _own(col_p.value, nnz, ctypes.c_int32, np.int32)
    return row_ptr, col


def erdos_renyi(n: int, m_edges: int, seed: int):
    """G(n, M): ``m_edges`` distinct undirected edges, uniform, no self-loops."""
    return _take(_load().sg_er(n, m_edges, seed))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, relabel: bool = True):
    """R-MAT with 2^scale vertices and edge_factor * 2^scale edge draws,
    symmetrised, deduplicated, self-loops dropped, vertices relabelled by a
    seeded random permutation.  d = 1 - a - b - c."""
    return _take(_load().sg_rmat(scale, edge_factor, a, b, c, seed, int(relabel)))


def rmat_pairs(scale: int, count: int, a: float = 0.57, b: float = 0.19, c: float = 0.19, seed: int = 1,
               relabel: bool = True, stream: int = 7, first: int = 0):
    """``count`` endpoint pairs drawn from the R-MAT distribution of
    ``rmat(scale, ..., seed)`` (same quadrant recursion, same relabelling),
    from counter stream ``stream`` starting at pair ``first``; self-loops
    included.  Returns an int64 array of shape (count, 2)."""
    u = np.empty(count, dtype=np.int32)
    v = np.empty(count, dtype=np.int32)
    if count:
        _load().sg_rmat_pairs(scale, a, b, c, seed, int(relabel), stream, first, count, u.ctypes.data, v.ctypes.data)
    return np.stack([u, v], 1).astype(np.int64)


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_LIB_PATH):
            raise RuntimeError(f"{_GPU_LIB_PATH} is not built; run synthgraph.build() first")
        lib = ctypes.CDLL(_GPU_LIB_PATH)
        vp = ctypes.c_void_p
        lib.sg_gpu_rmat_begin.restype = ctypes.c_int
        lib.sg_gpu_rmat_begin.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_uint64, vp, vp, ctypes.POINTER(vp),
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.sg_gpu_rmat_finish.restype = ctypes.c_int
        lib.sg_gpu_rmat_finish.argtypes = [vp, vp, vp]
        lib.sg_gpu_rmat_abort.restype = None
        lib.sg_gpu_rmat_abort.argtypes = [vp]
        _gpu_lib = lib
    return _gpu_lib


def rmat_device(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                c: float = 0.19, seed: int = 1, relabel: bool = True):
    """The graph of ``rmat`` (same arguments, bit for bit the same CSR), built
    on the current GPU: returns (row_ptr int64, col int32) torch tensors on
    that device.  For large scales (27: 4.3e9 arcs) this takes seconds where
    the host build takes minutes; it needs 16 bytes of device memory per arc
    draw while it runs."""
    import torch
    n = 1 << scale
    perm = None
    if relabel:
        perm = np.empty(n, dtype=np.int32)
        _load().sg_permutation(n, seed, perm.ctypes.data)
    lib = _load_gpu()
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(dev)
    handle = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    torch.cuda.synchronize(dev)
    rc = lib.sg_gpu_rmat_begin(scale, edge_factor, a, b, c, seed, perm.ctypes.data if perm is not None else None,
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(handle), ctypes.byref(nnz))
    if rc != 0:
        raise RuntimeError(f"GPU R-MAT build failed ({rc})")
    try:
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)[:nnz.value]
    except Exception:
        lib.sg_gpu_rmat_abort(handle)
        raise
    rc = lib.sg_gpu_rmat_finish(handle, ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col.data_ptr()))
    if rc != 0:
        raise RuntimeError(f"GPU R-MAT build failed ({rc})")
    return row_ptr, col


def rmat_directed(scale: int, edge_factor: int = 16, seed: int = 1, stream: int = 5):
    """Directed R-MAT: edge_factor * 2^scale arcs u -> v drawn from the R-MAT
    distribution of ``rmat(scale, seed=seed)`` (counter stream ``stream``),
    deduplicated, self-loops dropped; power-law out- and in-degrees that
    differ from node to node."""
    n = 1 << scale
    p = rmat_pairs(scale, edge_factor * n, seed=seed, stream=stream)
    return from_edges(n, p[:, 0], p[:, 1], undirected=False)


def barabasi_albert(n: int, m: int, seed: int):
    """Preferential attachment: (m+1)-clique seed, then m distinct targets per vertex."""
    return _take(_load().sg_ba(n, m, seed))


def raw_draws(seed: int, stream: int, first: int, count: int) -> np.ndarray:
    """The counter-based generator's 64-bit outputs, for pinning it in tests."""
    out = np.empty(count, dtype=np.uint64)
    _load().sg_draw(seed, stream, first, count, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Small fixed shapes (numpy), for tests.
# ---------------------------------------------------------------------------

def from_edges(n: int, src, dst, undirected: bool = True):
    """Canonical CSR from an arc list.  Undirected adds the reverse arcs.
    Self-loops and duplicates are removed; rows are sorted."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if undirected:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(src * n + dst)
    src, dst = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, dst.astype(np.int32)


def complete_graph(n: int):
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j)


def cycle_graph(n: int):
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n)


def star_graph(leaves: int):
    """Vertex 0 is the centre, vertices 1..leaves the leaves."""
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1))


def path_graph(n: int, undirected: bool = True):
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, undirected=undirected)


def random_graph(n: int, p: float, seed: int, undirected: bool = True):
    """Each pair (undirected) or ordered pair (directed) present with probability p."""
    rng = np.random.default_rng(seed)
    if undirected:
        i, j = np.triu_indices(n, 1)
        keep = rng.random(i.size) < p
        return from_edges(n, i[keep], j[keep], undirected=True)
    i, j = np.nonzero(rng.random((n, n)) < p)
    return from_edges(n, i, j, undirected=False)


def random_dag(n: int, p: float, seed: int):
    """Directed acyclic: arcs only from lower to higher id."""
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n, 1)
    keep = rng.random(i.size) < p
    return from_edges(n, i[keep], j[keep], undirected=False)


def with_isolated(row_ptr, col, extra: int):
    """Append ``extra`` isolated vertices."""
    tail = np.full(extra, row_ptr[-1], dtype=np.int64)
    return np.concatenate([row_ptr, tail]), col.copy()


def max_degree(row_ptr) -> int:
    row_ptr = np.asarray(row_ptr)
    return int(np.max(np.diff(row_ptr))) if row_ptr.size > 1 else 0
