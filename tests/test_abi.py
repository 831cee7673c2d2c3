"""The C ABI without a GPU: the library loads, exports every function that
include/katz.h declares, the binding's structs match the header's layout, and
argument errors come back before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "katz.h")


def K():
    import paper_1807_03847_amd.katz as katz
    return katz


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(katz_\w+)\s*\(", text, re.M)))


def test_header_functions_exported():
    names = declared_functions()
    assert {"katz_rank_static", "katz_rank_update", "katz_bounds", "katz_state_free",
            "katz_strerror"} <= set(names)
    lib = ctypes.CDLL(K().LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "katz.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("katz_csr %zu\nkatz_params %zu\nkatz_result %zu\nkatz_tuning %zu\nkatz_timing %zu\nkatz_solve_info %zu\n",
         sizeof(katz_csr), sizeof(katz_params), sizeof(katz_result), sizeof(katz_tuning), sizeof(katz_timing),
         sizeof(katz_solve_info));
  F(katz_csr, col) F(katz_csr, row_ptr_64) F(katz_csr, undirected)
  F(katz_params, k) F(katz_params, precision) F(katz_params, validate) F(katz_params, flags) F(katz_params, degree_cap)
  F(katz_params, criterion) F(katz_params, pair_u) F(katz_params, pair_v)
  F(katz_result, rest_upper_max) F(katz_result, active_final) F(katz_result, iterations) F(katz_result, status)
  F(katz_result, separated_fraction)
  F(katz_solve_info, converged) F(katz_solve_info, residual) F(katz_solve_info, alpha_used)
  F(katz_tuning, blocks_per_cu) F(katz_tuning, batch_blocks_per_cu) F(katz_tuning, batch_tile)
  F(katz_tuning, batch_xcd) F(katz_tuning, walk_groups) F(katz_tuning, split_hot_bytes) F(katz_tuning, bin_bounds)
  F(katz_tuning, reserved)
  F(katz_timing, prep_ms) F(katz_timing, calls) F(katz_timing, renumber_step_ms) F(katz_timing, renumber_step_launches)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split(" ") for line in out if line)
    katz = K()
    assert int(got["katz_csr"]) == ctypes.sizeof(katz.KatzCSR)
    assert int(got["katz_params"]) == ctypes.sizeof(katz.KatzParams)
    assert int(got["katz_result"]) == ctypes.sizeof(katz.KatzResult)
    assert int(got["katz_tuning"]) == ctypes.sizeof(katz.KatzTuning)
    assert int(got["katz_timing"]) == ctypes.sizeof(katz.KatzTiming)
    assert int(got["katz_solve_info"]) == ctypes.sizeof(katz.KatzSolveInfo)
    for key, val in got.items():
        if "." in key:
            struct, field = key.split(".")
            cls = {"katz_csr": katz.KatzCSR, "katz_params": katz.KatzParams, "katz_result": katz.KatzResult,
                   "katz_tuning": katz.KatzTuning, "katz_timing": katz.KatzTiming,
                   "katz_solve_info": katz.KatzSolveInfo}[struct]
            assert getattr(cls, field).offset == int(val), key


def test_strerror_covers_codes():
    katz = K()
    for code in range(-10, 4):
        assert "unknown" not in katz.strerror(code)
    assert "unknown" in katz.strerror(99)


def _call(g, p, res, count=1):
    katz = K()
    return katz.lib.katz_rank_static(count, ctypes.byref(g) if g is not None else None,
                                     ctypes.byref(p) if p is not None else None,
                                     ctypes.byref(res) if res is not None else None, None, None)


def test_argument_errors_before_device_work():
    katz = K()
    buf = (ctypes.c_int64 * 4)(0, 1, 2, 2)
    col = (ctypes.c_int32 * 2)(1, 0)
    out_ids = (ctypes.c_int32 * 8)()
    out_d = (ctypes.c_double * 8)()
    out_u = (ctypes.c_double * 8)()
    g = katz.KatzCSR(n=3, nnz=2, row_ptr=ctypes.addressof(buf), col=ctypes.addressof(col), row_ptr_64=1,
                     undirected=1)
    res = katz.KatzResult(topk_ids=ctypes.addressof(out_ids), lower=ctypes.addressof(out_d),
                          upper=ctypes.addressof(out_u))
    assert _call(g, katz.make_params(0), res) == katz.E_INVALID_ARG          # k < 1
    assert _call(g, katz.make_params(4), res) == katz.E_INVALID_ARG          # k > n
    assert _call(g, katz.make_params(1, alpha=float("nan")), res) == katz.E_ALPHA
    assert _call(g, katz.make_params(1, alpha=-1.0), res) == katz.E_ALPHA
    assert _call(g, katz.make_params(1, eps=-1.0), res) == katz.E_INVALID_ARG
    assert _call(g, katz.make_params(1, precision=7), res) == katz.E_INVALID_ARG
    p = katz.make_params(1)
    p.criterion = 9                                                      # unknown criterion
    assert _call(g, p, res) == katz.E_INVALID_ARG
    for pair in [(1, 1), (-1, 0), (0, 3), (3, 0)]:                      # equal or out-of-range pair ids
        assert _call(g, katz.make_params(1, criterion="pair", pair=pair), res) == katz.E_INVALID_ARG
    # Batches and states take the top-k criterion with k <= 4096 only.
    g2 = (katz.KatzCSR * 2)(g, g)
    p2 = (katz.KatzParams * 2)(katz.make_params(1, criterion="ranking"), katz.make_params(1, criterion="ranking"))
    r2 = (katz.KatzResult * 2)(res, res)
    assert katz.lib.katz_rank_static(2, g2, p2, r2, None, None) == katz.E_UNSUPPORTED
    st = (ctypes.c_void_p * 1)()
    assert katz.lib.katz_rank_static(1, ctypes.byref(g), ctypes.byref(katz.make_params(1, criterion="score")),
                                     ctypes.byref(res), st, None) == katz.E_UNSUPPORTED
    p = katz.make_params(1)
    p.flags = 1 << 7                                                     # unknown flag bit
    assert _call(g, p, res) == katz.E_INVALID_ARG
    assert _call(None, katz.make_params(1), res) == katz.E_INVALID_ARG
    assert _call(g, katz.make_params(1), res, count=0) == katz.E_INVALID_ARG
    bad = katz.KatzCSR(n=0, nnz=0, row_ptr=ctypes.addressof(buf), col=0, row_ptr_64=1, undirected=1)
    assert _call(bad, katz.make_params(1), res) == katz.E_INVALID_ARG
    lo = (ctypes.c_double * 3)()
    assert katz.lib.katz_bounds(ctypes.byref(g), ctypes.byref(katz.make_params(1)), 0, ctypes.addressof(lo),
                                ctypes.addressof(lo), None) == katz.E_INVALID_ARG
    assert katz.lib.katz_rank_update(None, None, None, 0, None, None, 0, None, None) == katz.E_INVALID_ARG
    info = katz.KatzSolveInfo()
    sc = (ctypes.c_double * 3)()
    pr = katz.make_params(1)
    assert katz.lib.katz_solve(ctypes.byref(g), ctypes.byref(pr), 5, 1e-9, ctypes.addressof(sc), ctypes.byref(info),
                               None) == katz.E_INVALID_ARG                  # unknown method
    assert katz.lib.katz_solve(ctypes.byref(g), ctypes.byref(pr), 0, 0.0, ctypes.addressof(sc), ctypes.byref(info),
                               None) == katz.E_INVALID_ARG                  # tol <= 0
    gd = katz.KatzCSR(n=3, nnz=2, row_ptr=ctypes.addressof(buf), col=ctypes.addressof(col), row_ptr_64=1,
                      undirected=0)
    assert katz.lib.katz_solve(ctypes.byref(gd), ctypes.byref(pr), katz.SOLVE_CG, 1e-9, ctypes.addressof(sc),
                               ctypes.byref(info), None) == katz.E_UNSUPPORTED  # CG needs a symmetric matrix


def test_tuning_round_trip_and_limits():
    katz = K()
    saved = katz.tuning_get()
    try:
        katz.tuning_set(16384, 4, 8, 2, 1)
        want = {"hub_bytes": 16384, "blocks_per_cu": 4, "batch_blocks_per_cu": 8, "batch_tile": 2, "batch_xcd": 1,
                "walk_groups": 0, "split_hot_bytes": 0, "bin_bounds": [0] * 6}
        assert katz.tuning_get() == want
        for bad in [(-16, 4, 0, 0), (65552, 4, 0, 0), (100, 4, 0, 0), (16384, 0, 0, 0),
                    (0, 33, 0, 0), (0, -1, 0, 0), (0, 0, 33, 0), (0, 0, -2, 0), (0, 0, 0, 17),
                    (0, 0, 0, -1), (0, 0, 0, 0, 2), (0, 0, 0, 0, -1), (0, 0, 0, 0, 0, 2), (0, 0, 0, 0, 0, 8),
                    (131072, 1, 0, 0, 0, 1), (162832, 1, 0, 0, 0, 4), (0, 0, 0, 0, 0, 0, -1),
                    (0, 0, 0, 0, 0, 0, 24), (0, 0, 0, 0, 0, 0, (64 << 20) + 16)]:
            with pytest.raises(katz.KatzError) as e:
                katz.tuning_set(*bad)
            assert e.value.code == katz.E_INVALID_ARG
            assert katz.tuning_get() == want                                  # unchanged
        katz.tuning_set(131072, 1, 0, 0, 0, 4)                              # large copy with 4 groups
        assert katz.tuning_get()["hub_bytes"] == 131072
        katz.tuning_set(0, 0, 0, 0, 0, 0, 1 << 20)                          # two-pass walk, 1 MiB hot set
        assert katz.tuning_get()["split_hot_bytes"] == 1 << 20
        katz.tuning_set(0, 0, 0, 0, 0, 0, 0)
        assert katz.tuning_get()["split_hot_bytes"] == 0
        # Row-length classes: all 0, or strictly increasing from 1 and below 4096.
        katz.tuning_set(bin_bounds=[2, 4, 8, 16, 64, 512])
        assert katz.tuning_get()["bin_bounds"] == [2, 4, 8, 16, 64, 512]
        for bad in ([0, 8, 16, 32, 128, 1024], [4, 4, 16, 32, 128, 1024], [4, 8, 16, 32, 1024, 128],
                    [4, 8, 16, 32, 128, 4096], [-1, 8, 16, 32, 128, 1024], [4, 0, 0, 0, 0, 0]):
            with pytest.raises(katz.KatzError) as e:
                katz.tuning_set(bin_bounds=bad)
            assert e.value.code == katz.E_INVALID_ARG
        assert katz.tuning_get()["bin_bounds"] == [2, 4, 8, 16, 64, 512]
        katz.tuning_set(16384, 4, 8, 2, 1)
        t = katz.KatzTuning(hub_bytes=0, blocks_per_cu=0)
        t.reserved = 1
        assert katz.lib.katz_tuning_set(ctypes.byref(t)) == katz.E_INVALID_ARG
        assert katz.lib.katz_tuning_set(None) == katz.E_INVALID_ARG
        assert katz.lib.katz_tuning_get(None) == katz.E_INVALID_ARG
        assert katz.lib.katz_autotune(1, None, None, None, None) == katz.E_INVALID_ARG
        assert katz.lib.katz_autotune(0, None, None, None, None) == katz.E_INVALID_ARG
    finally:
        katz.tuning_set(**saved)
