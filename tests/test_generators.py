"""Seeded input generators: determinism, canonical CSR form, counts."""
import numpy as np

import synthgraph as sg

MASK = (1 << 64) - 1


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def test_counter_generator_matches_splitmix64_definition():
    """The C generator is SplitMix64's finaliser over a Weyl sequence keyed by
    (seed, stream); recomputed here from that definition."""
    g = 0x9E3779B97F4A7C15
    for seed, stream in ((1, 1), (7, 3), (123456789, 2)):
        key = _mix((seed * g + _mix(stream + 0x632BE59BD9B4E019)) & MASK)
        want = [_mix((key + (i + 1) * g) & MASK) for i in range(5, 15)]
        got = sg.raw_draws(seed, stream, 5, 10)
        assert [int(v) for v in got] == want


def _canonical(rp, col, symmetric=True):
    n = len(rp) - 1
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size
    assert col.size == 0 or (col.min() >= 0 and col.max() < n)
    src = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(src == col)
    for v in range(0, n, max(1, n // 500)):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
    if symmetric:
        k1 = np.sort(src * n + col)
        k2 = np.sort(col.astype(np.int64) * n + src)
        assert np.array_equal(k1, k2)


def test_erdos_renyi_exact_count_and_determinism():
    rp, col = sg.erdos_renyi(16384, 131072, 1)
    assert rp[-1] == 262144
    _canonical(rp, col)
    rp2, col2 = sg.erdos_renyi(16384, 131072, 1)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    rp3, _ = sg.erdos_renyi(16384, 131072, 2)
    assert not np.array_equal(rp, rp3)


def test_rmat_canonical_and_deterministic():
    rp, col = sg.rmat(14, seed=3)
    _canonical(rp, col)
    rp2, col2 = sg.rmat(14, seed=3)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    n = 1 << 14
    # Dedup and loops remove some of the 2 * 16 * n directed draws, not most.
    assert 0.75 * 32 * n < rp[-1] <= 32 * n
    deg = np.diff(rp)
    assert deg.max() > 40 * deg[deg > 0].mean()     # heavy tail


def test_barabasi_albert_counts():
    n, m = 3000, 6
    rp, col = sg.barabasi_albert(n, m, 9)
    _canonical(rp, col)
    assert rp[-1] == 2 * (m * (m + 1) // 2 + (n - m - 1) * m)
    assert np.diff(rp).min() >= m


def test_small_shapes():
    rp, col = sg.complete_graph(5)
    assert np.all(np.diff(rp) == 4)
    rp, col = sg.star_graph(4)
    assert list(np.diff(rp)) == [4, 1, 1, 1, 1]
    rp, col = sg.path_graph(4, undirected=False)
    assert list(np.diff(rp)) == [1, 1, 1, 0]
    rp, col = sg.with_isolated(*sg.cycle_graph(3), 2)
    assert list(np.diff(rp)) == [2, 2, 2, 0, 0]


def test_rmat_pairs_follow_the_graph_distribution():
    """Pairs of counter stream 1 are the graph's own edge draws: every non-loop
    pair is an arc of rmat(scale, seed); another stream gives other pairs with
    the same skew (the graph's hubs are hit far more often than average)."""
    rp, col = sg.rmat(12, seed=4)
    n = len(rp) - 1
    keys = set((np.repeat(np.arange(n), np.diff(rp)) * n + col).tolist())
    own = sg.rmat_pairs(12, 20000, seed=4, stream=1)
    own = own[own[:, 0] != own[:, 1]]
    assert all(int(a) * n + int(b) in keys for a, b in own)
    other = sg.rmat_pairs(12, 20000, seed=4, stream=7)
    assert not np.array_equal(other[:100], sg.rmat_pairs(12, 100, seed=4, stream=1))
    hits = np.bincount(other.ravel(), minlength=n)
    deg = np.diff(rp)
    hubs = np.argsort(-deg)[:16]
    assert hits[hubs].mean() > 20 * hits.mean()
    assert np.array_equal(sg.rmat_pairs(12, 50, seed=4, stream=7, first=10), other[10:60])
