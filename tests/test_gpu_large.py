"""GPU parity at more than 2^31 arcs: R-MAT scale 27 (134M nodes, 4.2e9
directed entries, int64 row offsets), the large static workload, in both
forms, against the C++ form of the FP64 oracle on the host."""
import sys

import numpy as np
import pytest
import torch

import synthgraph as sg
from oracle import cpp as ocpp
from tests.parity import assert_topk_parity

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_rmat27_int64_offsets_against_oracle():
    import paper_1807_03847_amd.katz as katz
    say("rmat27 generate")
    rp_t, col_t = sg.rmat_device(27, 16, 0.57, 0.19, 0.19, seed=3)
    assert rp_t.dtype == torch.int64 and col_t.numel() > 2 ** 31
    say("rmat27 rank fp32 / fp64")
    r32 = katz.rank_static(rp_t, col_t, 100, eps=1e-6, precision="fp32")
    r64 = katz.rank_static(rp_t, col_t, 100, eps=1e-6, precision="fp64")
    torch.cuda.synchronize()
    say("rmat27 oracle")
    rp = rp_t.cpu().numpy()
    col = col_t.cpu().numpy()
    orc = ocpp.rank_static(rp, col, None, 100, 1e-6, full=True)
    del col
    for res, fp32 in ((r64, False), (r32, True)):
        assert_topk_parity(res.topk.cpu().numpy(), res.lower.cpu().numpy(), res.upper.cpu().numpy(), orc,
                           1e-12, widened=fp32, check_status=True, gpu_status=res.status)
    assert r64.iterations == orc.iterations
    assert abs(r64.rest_upper_max - orc.rest_upper_max) <= 1e-12 * orc.rest_upper_max
    # Scores at the oracle's r: every node's FP64 bounds (katz_bounds) within
    # 1e-12 relative of the oracle's, checked on a sample of a million nodes
    # and the whole top-100.
    say("rmat27 bounds")
    n = rp.size - 1
    lo_t, up_t = katz.bounds(rp_t, col_t, orc.iterations, precision="fp64")
    idx = np.unique(np.concatenate([np.random.default_rng(27).integers(0, n, 1 << 20), orc.topk]))
    it = torch.from_numpy(idx).cuda()
    lo, up = lo_t[it].cpu().numpy(), up_t[it].cpu().numpy()
    ol, ou = orc.lower_all[idx], orc.upper_all[idx]
    assert np.all(np.abs(lo - ol) <= 1e-12 * ol + 1e-300)
    assert np.all(np.abs(up - ou) <= 1e-12 * ou + 1e-300)
