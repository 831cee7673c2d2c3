"""katz_bounds with device outputs is stream-ordered and asynchronous: it
returns once its iterations are enqueued, its results equal the oracle's
once the stream completes, a call on another stream that reuses the
library's workspace is ordered after it, and a bad column id is still
reported by the call itself."""
import sys

import numpy as np
import pytest
import torch

import synthgraph as sg
from oracle import cpp as ocpp

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_bounds_async_on_two_streams():
    import paper_1807_03847_amd.katz as katz
    rp, col = sg.rmat(22, seed=1)
    rp_t = torch.from_numpy(rp).cuda()
    col_t = torch.from_numpy(col).cuda()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    say("async bounds r=30 on s1, r=5 on s2")
    with torch.cuda.stream(s1):
        lo1, up1 = katz.bounds(rp_t, col_t, 30)
        early = not s1.query()          # 30 walk steps of R-MAT 22 are still running
    with torch.cuda.stream(s2):
        lo2, up2 = katz.bounds(rp_t, col_t, 5)
    s1.synchronize()
    s2.synchronize()
    assert early
    for r, lo, up in ((30, lo1, up1), (5, lo2, up2)):
        olo, oup = ocpp.bounds(rp, col, None, r)
        glo, gup = lo.cpu().numpy(), up.cpu().numpy()
        assert np.all(np.abs(glo - olo) <= 1e-12 * olo + 1e-300)
        assert np.all(np.abs(gup - oup) <= 1e-12 * oup + 1e-300)


def test_bounds_async_reports_bad_columns():
    import paper_1807_03847_amd.katz as katz
    rp, col = sg.erdos_renyi(5000, 20000, 3)
    bad = col.copy()
    bad[len(bad) // 2] = 5000
    say("async bounds bad column")
    with pytest.raises(katz.KatzError) as e:
        katz.bounds(torch.from_numpy(rp).cuda(), torch.from_numpy(bad).cuda(), 4)
    assert e.value.code == katz.E_CSR
