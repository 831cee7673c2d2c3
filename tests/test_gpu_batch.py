"""GPU parity of the batched form (katz_rank_static with count > 1)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synthgraph as sg
from tests.parity import assert_topk_parity

pytestmark = pytest.mark.gpu


def K():
    import paper_1807_03847_amd.katz as katz
    return katz


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def batch_workload(count, seed, n_lo=10, n_hi=14):
    """Barabasi-Albert graphs with n log-uniform in [2^n_lo, 2^n_hi], m in 4..32,
    each with alpha = f/(1 + d_max), f in (0, 1], k in [10, 500] (capped at n/4)
    and eps = 1e-6 f."""
    rng = np.random.default_rng(seed)
    graphs, params = [], []
    for gidx in range(count):
        n = int(round(2 ** rng.uniform(n_lo, n_hi)))
        m = int(rng.integers(4, 33))
        m = min(m, n // 4)
        rp, col = sg.barabasi_albert(n, m, 1000 * seed + gidx + 1)
        f = float(rng.uniform(0.05, 1.0))
        alpha = f / (1 + sg.max_degree(rp))
        k = int(min(rng.integers(10, 501), n // 4))
        graphs.append((rp, col))
        params.append(dict(k=k, alpha=alpha, eps=1e-6 * f))
    return graphs, params


def run_batch(graphs, params, precision, host=False):
    katz = K()
    dev = (lambda a: torch.from_numpy(a)) if host else (lambda a: torch.from_numpy(a).cuda())
    gl = [(dev(np.asarray(rp, dtype=np.int64)), dev(np.asarray(col, dtype=np.int32)), True) for rp, col in graphs]
    pl = [dict(pp, precision=precision) for pp in params]
    return katz.rank_static_batch(gl, pl)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_single_and_oracle(precision):
    katz = K()
    graphs, params = batch_workload(24, 3)
    say("batch", precision, sum(len(rp) - 1 for rp, _ in graphs), "nodes")
    res = run_batch(graphs, params, precision)
    for (rp, col), pp, rb in zip(graphs, params, res):
        orc = oracle.rank_static(rp, col, pp["alpha"], pp["k"], pp["eps"])
        assert_topk_parity(rb.topk.cpu().numpy(), rb.lower.cpu().numpy(), rb.upper.cpu().numpy(), orc,
                           gpu_status=rb.status)
        single = katz.rank_static(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), pp["k"],
                                  alpha=pp["alpha"], eps=pp["eps"], precision=precision)
        assert torch.equal(single.topk, rb.topk)
        assert single.iterations == rb.iterations and single.status == rb.status
        if precision == "fp64":
            assert torch.equal(single.lower, rb.lower) and torch.equal(single.upper, rb.upper)
            assert single.rest_upper_max == rb.rest_upper_max


def circulant(n, offsets):
    src = np.concatenate([np.arange(n)] * len(offsets))
    dst = np.concatenate([(np.arange(n) + o) % n for o in offsets])
    return sg.from_edges(n, src, dst)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_all_nodes_tied(precision):
    """Vertex-transitive graphs: every node has the same bounds at every r, so
    the k-th key is shared by all n nodes, the selection breaks the tie by id
    over every node of the graph, and no ranking is ever certified (eps = 0:
    the iteration limit ends the run).  A BA graph in the same batch converges
    normally."""
    katz = K()
    graphs = [sg.cycle_graph(5000), sg.cycle_graph(70000), circulant(20000, (1, 5, 17)),
              sg.barabasi_albert(3000, 6, 77)]
    params = []
    for (rp, col), k in zip(graphs, (40, 700, 1000, 50)):
        params.append(dict(k=k, alpha=0.5 / (1 + sg.max_degree(rp)), eps=0.0, max_iter=9))
    params[-1]["eps"] = 1e-9
    say("batch all tied", precision)
    res = run_batch(graphs, params, precision)
    for gi, ((rp, col), pp, rb) in enumerate(zip(graphs, params, res)):
        orc = oracle.rank_static(rp, col, pp["alpha"], pp["k"], pp["eps"], max_iter=pp["max_iter"])
        if gi < 3:
            assert orc.status == oracle.W_ITER_LIMIT and rb.iterations == 9
        assert_topk_parity(rb.topk.cpu().numpy(), rb.lower.cpu().numpy(), rb.upper.cpu().numpy(), orc,
                           gpu_status=rb.status)
        single = katz.rank_static(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), pp["k"],
                                  alpha=pp["alpha"], eps=pp["eps"], precision=precision, max_iter=pp["max_iter"])
        assert torch.equal(single.topk, rb.topk)
        assert single.iterations == rb.iterations and single.status == rb.status
        if gi < 3:   # ties are broken by the smaller id: the k smallest ids, in order
            assert np.array_equal(rb.topk.cpu().numpy(), np.arange(pp["k"]))


def test_batch_uneven_convergence_and_host_buffers():
    """Graphs that stop at very different r (small alpha converges fast), host
    inputs and outputs, a graph with k = n."""
    graphs, params = batch_workload(6, 9, 10, 12)
    rp, col = sg.erdos_renyi(300, 900, 5)
    graphs.append((rp, col))
    params.append(dict(k=300, alpha=1.0 / (1 + sg.max_degree(rp)), eps=1e-9))
    params[0]["alpha"] *= 0.01
    say("batch uneven")
    res = run_batch(graphs, params, "fp64", host=True)
    iters = [r.iterations for r in res]
    assert max(iters) > min(iters)
    for (rp, col), pp, rb in zip(graphs, params, res):
        orc = oracle.rank_static(rp, col, pp["alpha"], pp["k"], pp["eps"])
        assert rb.iterations == orc.iterations
        assert_topk_parity(rb.topk.numpy(), rb.lower.numpy(), rb.upper.numpy(), orc, gpu_status=rb.status)
    assert res[-1].rest_upper_max == -np.inf


def test_batch_rejects_mixed_precision():
    katz = K()
    graphs, params = batch_workload(2, 1, 10, 10)
    gl = [(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), True) for rp, col in graphs]
    pl = [dict(params[0], precision="fp64"), dict(params[1], precision="fp32")]
    with pytest.raises(katz.KatzError) as e:
        katz.rank_static_batch(gl, pl)
    assert e.value.code == katz.E_UNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_long_rows_match_single(precision):
    """Rows longer than one 4096-arc segment (a star hub, R-MAT hubs) are summed
    in segments and combined per row; each graph's result equals the
    single-graph call bitwise."""
    katz = K()
    rp1, col1 = sg.star_graph(9000)
    rp2, col2 = sg.rmat(15, seed=21)
    rp3, col3 = sg.barabasi_albert(3000, 6, 22)
    graphs = [(rp1, col1), (rp2, col2), (rp3, col3)]
    assert sg.max_degree(rp1) > 8192 and sg.max_degree(rp2) > 4096
    params = [dict(k=min(50, len(rp) - 1), alpha=0.5 / (1 + sg.max_degree(rp)), eps=1e-7) for rp, _ in graphs]
    say("batch long rows", precision)
    res = run_batch(graphs, params, precision)
    for (rp, col), pp, rb in zip(graphs, params, res):
        single = katz.rank_static(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), pp["k"],
                                  alpha=pp["alpha"], eps=pp["eps"], precision=precision)
        assert torch.equal(single.topk, rb.topk)
        assert torch.equal(single.lower, rb.lower) and torch.equal(single.upper, rb.upper)
        assert single.iterations == rb.iterations and single.status == rb.status


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_launch_tuning_is_invisible(precision):
    """A persistent batched walk grid changes no result bit; the batch
    autotuner installs one of its candidates."""
    katz = K()
    graphs, params = batch_workload(10, 5)
    rp, col = sg.star_graph(5000)
    graphs.append((rp, col))
    params.append(dict(k=20, alpha=0.5 / (1 + sg.max_degree(rp)), eps=1e-7))
    saved = katz.tuning_get()
    try:
        katz.tuning_set(**dict(saved, batch_blocks_per_cu=0, batch_tile=0))
        ref = run_batch(graphs, params, precision)
        for bbpc, tile, xcd in ((1, 1, 0), (4, 3, 0), (32, 2, 0), (0, 16, 0), (0, 1, 1), (4, 3, 1), (32, 1, 1)):
            say("batch tuning", precision, bbpc, tile, xcd)
            katz.tuning_set(**dict(saved, batch_blocks_per_cu=bbpc, batch_tile=tile, batch_xcd=xcd))
            res = run_batch(graphs, params, precision)
            for a, b in zip(res, ref):
                assert torch.equal(a.topk, b.topk) and torch.equal(a.lower, b.lower) and torch.equal(a.upper, b.upper)
                assert (a.iterations, a.status) == (b.iterations, b.status)
        gl = [(torch.from_numpy(np.asarray(r, dtype=np.int64)).cuda(), torch.from_numpy(c).cuda(), True)
              for r, c in graphs]
        best = katz.autotune_batch(gl, [dict(pp, precision=precision) for pp in params])
        assert (best["batch_blocks_per_cu"], best["batch_tile"], best["batch_xcd"]) in (
            (0, 1, 0), (4, 1, 0), (16, 1, 0), (4, 2, 0), (16, 2, 0), (4, 4, 0), (16, 4, 0), (16, 8, 0), (0, 1, 1),
            (16, 1, 1), (4, 4, 1), (16, 4, 1), (16, 8, 1))
        assert katz.tuning_get() == best
    finally:
        katz.tuning_set(**saved)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_renumbering_is_invisible(precision):
    """Renaming each graph's nodes by its binned order changes only the memory
    layout: every output is bitwise that of the batch in caller order."""
    katz = K()
    graphs, params = batch_workload(8, 13)
    rp, col = sg.star_graph(6000)
    graphs.insert(3, (rp, col))
    params.insert(3, dict(k=25, alpha=0.5 / (1 + sg.max_degree(rp)), eps=1e-7))
    say("batch renumbering", precision)
    a = run_batch(graphs, [dict(pp, flags=katz.FLAG_REORDER) for pp in params], precision)
    b = run_batch(graphs, [dict(pp, flags=katz.FLAG_NO_REORDER) for pp in params], precision)
    for ra, rb in zip(a, b):
        assert torch.equal(ra.topk, rb.topk) and torch.equal(ra.lower, rb.lower) and torch.equal(ra.upper, rb.upper)
        assert (ra.iterations, ra.status, ra.rest_upper_max) == (rb.iterations, rb.status, rb.rest_upper_max)


def test_batch_column_errors():
    """A column id out of range in any graph (checked over the arcs of the whole
    batch in fixed-size chunks) fails the call."""
    katz = K()
    graphs, params = batch_workload(5, 17, 10, 12)
    for gi, pos in ((0, 0), (2, -1), (4, 777)):
        rp, col = graphs[gi]
        bad = col.copy()
        bad[pos] = len(rp) - 1 + 3
        gl = list(graphs)
        gl[gi] = (rp, bad)
        say("batch column error", gi, pos)
        with pytest.raises(katz.KatzError) as e:
            run_batch(gl, params, "fp64")
        assert e.value.code == katz.E_CSR
    res = run_batch(graphs, params, "fp64")
    assert len(res) == len(graphs)


def test_batch_graph_replayed_across_calls():
    """A batch of the same shape in the same workspace replays the hipGraph the
    previous call instantiated: three calls on one batch, a different batch in
    between (re-captured), and the first batch again all give bitwise the same
    results as its first call; every result is the oracle's."""
    katz = K()
    g1, p1 = batch_workload(12, 7)
    g2, p2 = batch_workload(9, 8)
    say("batch graph replay")
    dev = lambda a: torch.from_numpy(a).cuda()
    gl1 = [(dev(np.asarray(rp, dtype=np.int64)), dev(np.asarray(col, dtype=np.int32)), True) for rp, col in g1]
    gl2 = [(dev(np.asarray(rp, dtype=np.int64)), dev(np.asarray(col, dtype=np.int32)), True) for rp, col in g2]
    pl1 = [dict(pp, precision="fp32") for pp in p1]
    pl2 = [dict(pp, precision="fp32") for pp in p2]
    first = katz.rank_static_batch(gl1, pl1)
    runs = [katz.rank_static_batch(gl1, pl1), katz.rank_static_batch(gl1, pl1)]
    other = katz.rank_static_batch(gl2, pl2)
    runs.append(katz.rank_static_batch(gl1, pl1))
    for res in runs:
        for a, b in zip(res, first):
            assert torch.equal(a.topk, b.topk) and torch.equal(a.lower, b.lower) and torch.equal(a.upper, b.upper)
            assert (a.iterations, a.status) == (b.iterations, b.status)
    for (rp, col), pp, rb in list(zip(g1, p1, first)) + list(zip(g2, p2, other)):
        orc = oracle.rank_static(rp, col, pp["alpha"], pp["k"], pp["eps"])
        assert_topk_parity(rb.topk.cpu().numpy(), rb.lower.cpu().numpy(), rb.upper.cpu().numpy(), orc,
                           widened=True, check_status=False)
