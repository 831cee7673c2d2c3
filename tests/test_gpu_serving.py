"""Serving form: each request's result is the same alone and in the mix."""
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


def request_stream(rp, col, n, count, rng, max_batch=60, hubs=()):
    """`count` valid batches applied in order: 70% insertions of absent edges,
    30% deletions of present ones (undirected pairs a < b)."""
    src = np.repeat(np.arange(n), np.diff(rp))
    edges = set(zip(src[src < col].tolist(), col[src < col].tolist()))
    out = []
    for _ in range(count):
        size = int(rng.integers(1, max_batch + 1))
        n_ins = max(1, int(round(0.7 * size)))
        n_del = size - n_ins
        dels = [tuple(e) for e in rng.permutation(sorted(edges))[:n_del].tolist()] if n_del else []
        ins = set()
        while len(ins) < n_ins:
            a = int(rng.choice(hubs)) if len(hubs) and rng.random() < 0.3 else int(rng.integers(0, n))
            b = int(rng.integers(0, n))
            a, b = min(a, b), max(a, b)
            if a != b and (a, b) not in edges and (a, b) not in ins:
                ins.add((a, b))
        for e in dels:
            edges.discard(e)
        edges |= ins
        out.append((np.array(sorted(ins), dtype=np.int64).reshape(-1, 2),
                    np.array(dels, dtype=np.int64).reshape(-1, 2)))
    return out


def make_graphs():
    gs = [sg.erdos_renyi(2000, 8000, 3), sg.rmat(12, seed=4), sg.barabasi_albert(3000, 5, 6)]
    out = []
    for rp, col in gs:
        dmax = sg.max_degree(rp)
        H = 200
        out.append((rp, col, 1.0 / (1 + dmax + H), dmax + H))
    return out


@pytest.mark.parametrize("slots,budget,late_add", [(3, 0, False), (2, 1, False), (3, 0, True)])
def test_serving_mix_equals_alone(slots, budget, late_add):
    """late_add: graphs after the first are registered while the first graph's
    requests run, so the server's graph table grows under running workers."""
    katz = K()
    rng = np.random.default_rng(slots)
    graphs = make_graphs()
    k, eps = 25, 1e-9
    streams = []
    for rp, col, alpha, cap in graphs:
        hubs = np.argsort(-np.diff(rp))[:5]
        streams.append(request_stream(rp, col, len(rp) - 1, 8, rng, hubs=hubs))
    say("serving mix", slots, budget, late_add)
    sv = katz.Server(slots=slots, memory_budget=budget)
    gids = []
    tickets = []
    for gi, (rp, col, alpha, cap) in enumerate(graphs):
        gid, _ = sv.add_graph(torch.from_numpy(rp), torch.from_numpy(col), k, alpha=alpha, eps=eps, degree_cap=cap)
        gids.append(gid)
        if late_add and gi == 0:
            tickets += [(0, j, sv.submit(gid, *streams[0][j])) for j in range(8)]
    for j in range(8):                      # interleave the graphs' requests
        for gi, gid in enumerate(gids):
            if late_add and gi == 0:
                continue
            ins, dels = streams[gi][j]
            tickets.append((gi, j, sv.submit(gid, ins, dels)))
    mixed = {}
    for gi, j, t in tickets:
        res, lat, svc = sv.wait(t)
        assert lat >= svc > 0
        mixed[(gi, j)] = res
    sv.close()
    # Every mixed result against the oracle's Algorithm 2 replaying the same
    # per-graph request sequence (delta form, FP64 on the host).
    say("serving oracle")
    for gi, (rp, col, alpha, cap) in enumerate(graphs):
        dyn = oracle.DynamicOracle(rp, col, alpha, k=k, eps=eps, degree_cap=cap)
        for j, (ins, dels) in enumerate(streams[gi]):
            orc = dyn.update(ins, dels)
            m = mixed[(gi, j)]
            assert m.iterations == orc.iterations
            assert_topk_parity(m.topk, m.lower, m.upper, orc, gpu_status=m.status)
    say("serving alone")
    for gi, (rp, col, alpha, cap) in enumerate(graphs):
        st, _ = katz.create_state(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), k, alpha=alpha,
                                  eps=eps, degree_cap=cap)
        for j, (ins, dels) in enumerate(streams[gi]):
            alone = st.update(ins, dels)
            m = mixed[(gi, j)]
            assert np.array_equal(alone.topk.cpu().numpy(), m.topk)
            assert np.array_equal(alone.lower.cpu().numpy(), m.lower)
            assert np.array_equal(alone.upper.cpu().numpy(), m.upper)
            assert (alone.iterations, alone.status) == (m.iterations, m.status)
        st.free()


def test_serving_reports_errors_per_request():
    katz = K()
    rp, col = sg.erdos_renyi(500, 2000, 8)
    sv = katz.Server(slots=2)
    gid, _ = sv.add_graph(torch.from_numpy(rp), torch.from_numpy(col), 10, alpha=1.0 / (2 + sg.max_degree(rp)),
                          eps=1e-9, degree_cap=sg.max_degree(rp) + 1)
    src = np.repeat(np.arange(500), np.diff(rp))
    t_bad = sv.submit(gid, np.array([[src[0], col[0]]]), None)       # already present
    with pytest.raises(katz.KatzError) as e:
        sv.wait(t_bad)
    assert e.value.code == katz.E_UPDATE
    sv.close()


def test_destroy_cancels_queued_requests():
    """Destroying a server with requests still queued: threads blocked in
    wait return (the request ran, or E_CANCELLED), and destroy returns once
    they have.  A first request of 200000 edges keeps the single slot busy
    while the others queue."""
    import threading
    import time
    katz = K()
    rng = np.random.default_rng(5)
    rp, col = sg.rmat(20, seed=9)
    dmax = sg.max_degree(rp)
    n = len(rp) - 1
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp)) * n + col

    def fresh_pairs(count):
        a = rng.integers(0, n, 3 * count)
        b = rng.integers(0, n, 3 * count)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        k = np.unique(lo * n + hi)
        pos = np.minimum(np.searchsorted(keys, k), keys.size - 1)
        k = k[(keys[pos] != k) & (k // n != k % n)]
        k = rng.permutation(k)[:count]
        return np.stack([k // n, k % n], 1)

    pairs = fresh_pairs(200000 + 30 * 50)
    stream = [(pairs[:200000], None)] + [(pairs[200000 + 50 * j:200000 + 50 * (j + 1)], None) for j in range(30)]
    say("serving destroy")
    sv = katz.Server(slots=1)
    gid, _ = sv.add_graph(torch.from_numpy(rp), torch.from_numpy(col), 20, alpha=1.0 / (1 + dmax + 1000),
                          eps=1e-9, degree_cap=dmax + 1000)
    tickets = [sv.submit(gid, ins, dels) for ins, dels in stream]
    codes = {}

    def waiter(t):
        try:
            codes[t] = sv.wait(t)[0].status
        except katz.KatzError as e:
            codes[t] = e.code

    threads = [threading.Thread(target=waiter, args=(t,)) for t in tickets[-6:]]
    for th in threads:
        th.start()
    time.sleep(0.05)      # the waiters are inside katz_server_wait (no call may start after destroy)
    sv.close()
    for th in threads:
        th.join(timeout=120)
        assert not th.is_alive()
    assert set(codes) == set(tickets[-6:])
    assert all(c in (katz.OK, katz.E_CANCELLED) for c in codes.values())
    assert katz.E_CANCELLED in codes.values()


def test_cancel_and_timed_wait():
    """katz_server_cancel ends a request that has not reached the device (its
    waiter gets E_CANCELLED and later requests of the graph run without its
    batch); a timed wait on unfinished work returns E_TIMEOUT and leaves the
    ticket valid; a finished or running request cannot be cancelled.  A first
    request of 200000 edges keeps the single slot busy meanwhile."""
    katz = K()
    rng = np.random.default_rng(11)
    rp, col = sg.rmat(20, seed=9)
    dmax = sg.max_degree(rp)
    n = len(rp) - 1
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp)) * n + col
    a = rng.integers(0, n, 700000)
    b = rng.integers(0, n, 700000)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    kk = np.unique(lo * n + hi)
    pos = np.minimum(np.searchsorted(keys, kk), keys.size - 1)
    kk = rng.permutation(kk[(keys[pos] != kk) & (kk // n != kk % n)])
    pairs = np.stack([kk // n, kk % n], 1)
    big, b1, b2, b3 = pairs[:200000], pairs[200000:200040], pairs[200040:200080], pairs[200080:200120]
    alpha = 1.0 / (1 + dmax + 1000)
    say("serving cancel")
    sv = katz.Server(slots=1)
    gid, _ = sv.add_graph(torch.from_numpy(rp), torch.from_numpy(col), 20, alpha=alpha, eps=1e-9,
                          degree_cap=dmax + 1000)
    t0 = sv.submit(gid, big, None)
    t1 = sv.submit(gid, b1, None)
    t2 = sv.submit(gid, b2, None)
    t3 = sv.submit(gid, b3, None)
    with pytest.raises(katz.KatzError) as e:
        sv.wait(t0, timeout_ms=0)                      # the big batch is still running
    assert e.value.code == katz.E_TIMEOUT
    assert sv.cancel(t2) == katz.OK
    with pytest.raises(katz.KatzError) as e:
        sv.cancel(t2)                                  # already ended
    assert e.value.code == katz.E_BUSY
    r0, _, _ = sv.wait(t0)
    r1, _, _ = sv.wait(t1)
    with pytest.raises(katz.KatzError) as e:
        sv.wait(t2)
    assert e.value.code == katz.E_CANCELLED
    r3, _, _ = sv.wait(t3, timeout_ms=600000)
    with pytest.raises(katz.KatzError) as e:
        sv.cancel(t3)                                  # collected: unknown ticket
    assert e.value.code == katz.E_INVALID_ARG
    sv.close()
    # The same sequence without the cancelled batch, on a state of its own.
    st, _ = katz.create_state(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), 20, alpha=alpha, eps=1e-9,
                              degree_cap=dmax + 1000)
    for got, batch in ((r0, big), (r1, b1), (r3, b3)):
        ref = st.update(batch, None)
        np.testing.assert_array_equal(np.asarray(got.topk), ref.topk.cpu().numpy())
        np.testing.assert_array_equal(np.asarray(got.lower), ref.lower.cpu().numpy())
    st.free()
