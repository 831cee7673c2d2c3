"""GPU parity of the inbound form (KATZ_FLAG_INBOUND): inbound Katz centrality is
the outbound centrality of the reverse graph (Section 2.1), which the library
builds on the device with a stable radix transpose.

The oracle ranks its own reverse graph (``oracle.reverse_graph``, a plain numpy
sort).  Because the device transpose lists every reversed row's sources in
ascending order, an inbound call must also be bitwise the outbound call on a
reverse graph that the caller built: that pins the transpose itself (rows,
offsets, order) at sizes that take one, two and three radix passes and span
many tiles."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synthgraph as sg
from tests.parity import assert_topk_parity

pytestmark = pytest.mark.gpu

TAU = 1e-12


def K():
    import paper_1807_03847_amd.katz as katz
    return katz


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(rp, col, rp64=True):
    rp_t = torch.from_numpy(np.asarray(rp, dtype=np.int64 if rp64 else np.int32)).cuda()
    col_t = torch.from_numpy(np.asarray(col, dtype=np.int32)).cuda()
    return rp_t, col_t


def graphs():
    """Directed graphs: n <= 256 (one radix pass), n = 4096 (two passes of 6
    bits), n = 2^17 (three passes), with empty rows and hubs."""
    out = []
    out.append(("dag40", sg.random_dag(40, 0.2, 5)))
    out.append(("rand200", sg.random_graph(200, 0.05, 9, undirected=False)))
    out.append(("rmatd12", sg.rmat_directed(12, 8, seed=2)))
    out.append(("rmatd17", sg.rmat_directed(17, 8, seed=4)))
    rp, col = sg.rmat_directed(10, 4, seed=6)
    out.append(("rmatd10_isolated_tail", sg.with_isolated(rp, col, 300)))
    return out


@pytest.mark.parametrize("name,g", graphs())
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inbound_topk_matches_oracle_on_reverse_graph(name, g, precision):
    say("inbound topk", name, precision)
    rp, col = g
    rt, rc = oracle.reverse_graph(rp, col)
    dmax = sg.max_degree(rt)
    alpha = 1.0 / (1 + dmax)
    n = len(rp) - 1
    k = min(50, n)
    eps = 1e-9 if precision == "fp64" else 1e-6
    orc = oracle.rank_static(rt, rc, alpha, k, eps, undirected=False)
    rp_t, col_t = dev(rp, col)
    res = K().rank_static(rp_t, col_t, k, alpha=alpha, eps=eps, precision=precision, undirected=False,
                          flags=K().FLAG_INBOUND)
    torch.cuda.synchronize()
    if precision == "fp32" and res.status == K().W_PRECISION_LIMIT:
        pytest.xfail("eps below the FP32 rounding margin")
    assert_topk_parity(res.topk.cpu().numpy(), res.lower.cpu().numpy(), res.upper.cpu().numpy(), orc, TAU,
                       widened=precision == "fp32", check_status=True, gpu_status=res.status)
    assert res.alpha == alpha


@pytest.mark.parametrize("name,g", graphs())
def test_inbound_is_bitwise_the_outbound_run_on_the_reverse_graph(name, g):
    """The device transpose is the oracle's reverse graph exactly: ids, bounds,
    r and status of the inbound call equal, bit for bit, those of an outbound
    call on the reverse graph built on the host."""
    say("inbound bitwise", name)
    rp, col = g
    rt, rc = oracle.reverse_graph(rp, col)
    n = len(rp) - 1
    k = min(40, n)
    rp_t, col_t = dev(rp, col, rp64=False)
    rt_t, rc_t = dev(rt, rc)
    for precision in ("fp64", "fp32"):
        a = K().rank_static(rp_t, col_t, k, eps=1e-7, precision=precision, undirected=False, flags=K().FLAG_INBOUND)
        b = K().rank_static(rt_t, rc_t, k, eps=1e-7, precision=precision, undirected=False)
        torch.cuda.synchronize()
        assert torch.equal(a.topk, b.topk)
        assert torch.equal(a.lower, b.lower) and torch.equal(a.upper, b.upper)
        assert (a.iterations, a.status, a.alpha) == (b.iterations, b.status, b.alpha)
    lo_a, up_a = K().bounds(rp_t, col_t, 4, undirected=False, flags=K().FLAG_INBOUND)
    lo_b, up_b = K().bounds(rt_t, rc_t, 4, undirected=False)
    torch.cuda.synchronize()
    assert torch.equal(lo_a, lo_b) and torch.equal(up_a, up_b)


def test_inbound_bounds_and_foster_match_oracle():
    say("inbound bounds and foster")
    rp, col = sg.rmat_directed(14, 8, seed=8)
    rt, rc = oracle.reverse_graph(rp, col)
    alpha = 1.0 / (1 + sg.max_degree(rt))
    rp_t, col_t = dev(rp, col)
    for r in (1, 3, 6):
        lo, up = K().bounds(rp_t, col_t, r, alpha=alpha, undirected=False, flags=K().FLAG_INBOUND)
        olo, oup = oracle.bounds(rt, rc, alpha, r, undirected=False)
        np.testing.assert_allclose(lo.cpu().numpy(), olo, rtol=1e-12, atol=0)
        np.testing.assert_allclose(up.cpu().numpy(), oup, rtol=1e-12, atol=0)
    scores, info, rc_ = K().solve(rp_t, col_t, "foster", 1e-9, alpha=alpha, undirected=False,
                                  flags=K().FLAG_INBOUND)
    orc = oracle.foster(rt, rc, alpha, 1e-9)
    assert info["iterations"] == orc.iterations
    np.testing.assert_allclose(scores.cpu().numpy(), orc.scores, rtol=1e-12, atol=0)


def test_inbound_from_host_memory_and_int32_offsets():
    say("inbound host inputs")
    rp, col = sg.rmat_directed(11, 8, seed=3)
    rt, rc = oracle.reverse_graph(rp, col)
    k = 30
    rp_h = torch.from_numpy(np.asarray(rp, dtype=np.int32))
    col_h = torch.from_numpy(np.asarray(col, dtype=np.int32))
    out = tuple(t.cuda() for t in (torch.empty(k, dtype=torch.int32), torch.empty(k, dtype=torch.float64),
                                   torch.empty(k, dtype=torch.float64)))
    a = K().rank_static(rp_h, col_h, k, eps=1e-8, undirected=False, flags=K().FLAG_INBOUND, out=out)
    rt_t, rc_t = dev(rt, rc)
    b = K().rank_static(rt_t, rc_t, k, eps=1e-8, undirected=False)
    torch.cuda.synchronize()
    assert torch.equal(a.topk, b.topk) and torch.equal(a.lower, b.lower)


def test_inbound_edge_cases():
    say("inbound edge cases")
    katz = K()
    # No arcs at all: every bound is zero, the ranking is by id.
    rp = np.zeros(9, dtype=np.int64)
    col = np.zeros(0, dtype=np.int32)
    rp_t, col_t = dev(rp, col)
    res = katz.rank_static(rp_t, col_t, 3, alpha=0.5, undirected=False, flags=katz.FLAG_INBOUND)
    torch.cuda.synchronize()
    assert res.topk.cpu().tolist() == [0, 1, 2]
    assert float(res.upper.max()) == 0.0
    # An undirected graph is its own reverse: the flag changes nothing.
    rp, col = sg.erdos_renyi(3000, 9000, 5)
    rp_t, col_t = dev(rp, col)
    a = katz.rank_static(rp_t, col_t, 20, eps=1e-9, flags=katz.FLAG_INBOUND)
    b = katz.rank_static(rp_t, col_t, 20, eps=1e-9)
    torch.cuda.synchronize()
    assert torch.equal(a.topk, b.topk) and torch.equal(a.lower, b.lower)
    # A column id out of range is an error before the transpose places any arc.
    rp, col = sg.rmat_directed(8, 4, seed=1)
    bad = np.array(col, copy=True)
    bad[len(bad) // 2] = len(rp) - 1
    rp_t, col_t = dev(rp, bad)
    with pytest.raises(katz.KatzError) as e:
        katz.rank_static(rp_t, col_t, 5, undirected=False, flags=katz.FLAG_INBOUND,
                         validate=katz.VALIDATE_NONE)
    assert e.value.code == katz.E_CSR
    # The allocation-free entry point does not take it.
    rp, col = sg.rmat_directed(8, 4, seed=1)
    rp_t, col_t = dev(rp, col)
    with pytest.raises(katz.KatzError) as e:
        katz.rank_static_noalloc(rp_t, col_t, 3, undirected=False, flags=katz.FLAG_INBOUND)
    assert e.value.code == katz.E_UNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inbound_in_a_batch_is_bitwise_the_single_call(precision):
    """A batch mixing inbound, outbound directed and undirected graphs: each
    result is bitwise the single-graph call with the same flags, and the
    inbound ones match the oracle on their reverse graphs."""
    katz = K()
    specs = [(sg.rmat_directed(11, 8, seed=1), False, katz.FLAG_INBOUND),
             (sg.rmat_directed(12, 6, seed=2), False, 0),
             (sg.rmat(11, seed=3), True, 0),
             (sg.rmat_directed(10, 8, seed=4), False, katz.FLAG_INBOUND)]
    eps = 1e-7 if precision == "fp64" else 1e-6
    graphs, params = [], []
    for (rp, col), und, flags in specs:
        graphs.append((*dev(rp, col), und))
        params.append(dict(k=25, eps=eps, precision=precision, flags=flags))
    say("inbound batch", precision)
    outs = katz.rank_static_batch(graphs, params)
    for ((rp, col), und, flags), (rp_t, col_t, _), res in zip(specs, graphs, outs):
        one = katz.rank_static(rp_t, col_t, 25, eps=eps, precision=precision, undirected=und, flags=flags)
        assert torch.equal(res.topk, one.topk) and torch.equal(res.lower, one.lower)
        assert torch.equal(res.upper, one.upper) and res.iterations == one.iterations
        if flags:
            rt, rc = oracle.reverse_graph(rp, col)
            orc = oracle.rank_static(rt, rc, 1.0 / (1 + sg.max_degree(rt)), 25, eps, undirected=False)
            assert_topk_parity(res.topk.cpu().numpy(), res.lower.cpu().numpy(), res.upper.cpu().numpy(), orc,
                               TAU, widened=precision == "fp32", gpu_status=res.status)
