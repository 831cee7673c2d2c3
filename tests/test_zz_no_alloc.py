"""katz_rank_static_noalloc (the entry point that allocates nothing) against
katz_rank_static, through the C ABI: bitwise-equal results on consecutive
calls, the second with a smaller graph, with device and host outputs, and a
clear error for a graph whose workspace exceeds the fixed scratch array."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import synthgraph as sg

pytestmark = pytest.mark.gpu


def K():
    import paper_1807_03847_amd.katz as katz
    return katz


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def call(entry, rp_t, col_t, k, eps, precision, host_out=False):
    katz = K()
    g = katz.make_csr(rp_t, col_t)
    p = katz.make_params(k, 0.0, eps, precision)
    dev = "cpu" if host_out else "cuda"
    ids = torch.full((k,), -1, dtype=torch.int32, device=dev)
    lo = torch.full((k,), -1.0, dtype=torch.float64, device=dev)
    up = torch.full((k,), -1.0, dtype=torch.float64, device=dev)
    res = katz.KatzResult(topk_ids=ids.data_ptr(), lower=lo.data_ptr(), upper=up.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if entry == "noalloc":
        rc = katz.lib.katz_rank_static_noalloc(ctypes.byref(g), ctypes.byref(p), ctypes.byref(res), stream)
    else:
        rc = katz.lib.katz_rank_static(1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(res), None, stream)
    torch.cuda.synchronize()
    return rc, res, ids.cpu(), lo.cpu(), up.cpu()


def same(a, b):
    rc_a, ra, ia, la, ua = a
    rc_b, rb, ib, lb, ub = b
    assert rc_a == rc_b >= 0
    assert torch.equal(ia, ib) and torch.equal(la, lb) and torch.equal(ua, ub)
    for f in ("iterations", "status", "active_final", "rest_upper_max", "alpha_used", "eta"):
        assert getattr(ra, f) == getattr(rb, f), f


@pytest.mark.parametrize("precision,eps", [("fp64", 0.0), ("fp32", 1e-6)])
def test_noalloc_matches_rank_static(precision, eps):
    cases = [(sg.rmat(15, 16, seed=7), 500), (sg.erdos_renyi(3000, 24000, 4), 64)]   # second one smaller
    for (rp, col), k in cases:
        say("noalloc", precision, "n", len(rp) - 1, "k", k)
        rp_t = torch.from_numpy(rp).cuda()
        col_t = torch.from_numpy(col).cuda()
        ref = call("static", rp_t, col_t, k, eps, precision)
        got = call("noalloc", rp_t, col_t, k, eps, precision)
        same(got, ref)
        same(call("noalloc", rp_t, col_t, k, eps, precision, host_out=True), ref)


def test_noalloc_rejects_oversize_then_still_works():
    katz = K()
    say("noalloc oversize")
    rp, col = sg.rmat(20, 16, seed=1)
    rp_t = torch.from_numpy(rp).cuda()
    col_t = torch.from_numpy(col).cuda()
    rc, *_ = call("noalloc", rp_t, col_t, 100, 1e-6, "fp32")
    assert rc == katz.E_SCRATCH
    assert "scratch" in katz.strerror(rc)
    rp, col = sg.erdos_renyi(2000, 16000, 5)
    rp_t = torch.from_numpy(rp).cuda()
    col_t = torch.from_numpy(col).cuda()
    same(call("noalloc", rp_t, col_t, 50, 0.0, "fp64"), call("static", rp_t, col_t, 50, 0.0, "fp64"))
