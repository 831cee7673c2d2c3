"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the FP64 oracle (``oracle.katz``) or its exact counterpart
(``oracle.exact``) against something that is not the oracle itself: closed forms,
brute-force enumeration, the pairwise definition of the top-k criterion, dense
linear algebra, or a different algorithmic route (Foster's recurrence, static
recomputation after a dynamic update).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from oracle import katz as K
import synthgraph as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
ULP = 2.0 ** -52


def small_graphs():
    """Tiny graphs of several shapes, undirected and directed."""
    out = []
    for seed in range(12):
        n = 4 + seed % 5
        out.append(("und", sg.random_graph(n, 0.45, seed), True))
        out.append(("dir", sg.random_graph(n, 0.35, 100 + seed, undirected=False), False))
    out.append(("star", sg.star_graph(5), True))
    out.append(("path", sg.path_graph(6), True))
    out.append(("cycle", sg.cycle_graph(7), True))
    out.append(("dag", sg.random_dag(7, 0.4, 3), False))
    return out


def _nonempty(rp):
    return sg.max_degree(rp) > 0


# --- walk counts -------------------------------------------------------------

@pytest.mark.parametrize("name,g,und", small_graphs())
def test_walk_recurrence_matches_enumeration(name, g, und):
    """x_i / alpha^i equals the number of walks of length i found by enumeration."""
    rp, col = g
    if not _nonempty(rp):
        pytest.skip("no arcs")
    dmax = sg.max_degree(rp)
    alpha = 1.0 / (1 + dmax)
    A = K.adjacency(rp, col)
    x = np.ones(len(rp) - 1)
    for i in range(1, 7):
        x = K.walk_step(A, x, alpha)
        want = np.array(exact.walks_bruteforce(rp, col, i), dtype=np.float64)
        np.testing.assert_allclose(x / alpha ** i, want, rtol=8 * i * ULP)


def test_regular_graph_walks_are_powers():
    """On a d-regular graph omega_i = d^i for every node."""
    rp, col = sg.cycle_graph(11)
    A = K.adjacency(rp, col)
    x = np.ones(11)
    for i in range(1, 20):
        x = K.walk_step(A, x, 1.0)   # alpha = 1 exposes omega directly
        assert np.all(x == 2.0 ** i)


# --- closed forms ---------------------------------------------------------------

def _golden_graph(case):
    if case["graph"] == "complete":
        return sg.complete_graph(case["n"]), True
    if case["graph"] == "cycle":
        return sg.cycle_graph(case["n"]), True
    if case["graph"] == "star":
        return sg.star_graph(case["leaves"]), True
    if case["graph"] == "path_directed":
        return sg.path_graph(case["n"], undirected=False), False
    raise KeyError(case["graph"])


def _golden_expected(case, n):
    if case["node"] == "all":
        vals = case["katz"] if isinstance(case["katz"], list) else [case["katz"]] * n
        return [Fraction(v) for v in vals]
    if case["node"] == "centre":
        return {0: Fraction(case["katz"])}
    return {v: Fraction(case["katz"]) for v in range(1, n)}


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["graph"])
def test_closed_forms_exact(case):
    """Rational Gaussian elimination of Eq. (la) reproduces the hand-derived values."""
    (rp, col), _ = _golden_graph(case)
    n = len(rp) - 1
    c = exact.katz_exact(rp, col, Fraction(case["alpha"]))
    want = _golden_expected(case, n)
    items = enumerate(want) if isinstance(want, list) else want.items()
    for v, val in items:
        assert c[v] == val


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["graph"])
def test_closed_forms_bracketed_by_oracle_bounds(case):
    """Every oracle iterate brackets the closed-form score; the bounds close on it."""
    (rp, col), und = _golden_graph(case)
    n = len(rp) - 1
    alpha = float(Fraction(case["alpha"]))
    want = _golden_expected(case, n)
    items = list(enumerate(want)) if isinstance(want, list) else list(want.items())
    for r in range(1, 60):
        lo, up = oracle.bounds(rp, col, alpha, r, undirected=und)
        for v, val in items:
            cv = float(val)
            tol = 8 * r * ULP * max(cv, 1e-300)
            assert lo[v] <= cv + tol and cv - tol <= up[v], (r, v)
    lo, up = oracle.bounds(rp, col, alpha, 400, undirected=und)
    for v, val in items:
        assert abs(lo[v] - float(val)) <= 1e-12 * max(1.0, float(val))


@pytest.mark.parametrize("n", [4, 6, 9])
def test_sharpness_complete_graph(n):
    """Appendix A: on K_n the upper bound equals the Katz score at every iteration."""
    rp, col = sg.complete_graph(n)
    alpha = 1.0 / n          # = 1/(1 + deg_max)
    cval = (n - 1.0)         # delta/(1-delta) with delta = (n-1)/n
    for r in range(1, 30):
        _, up = oracle.bounds(rp, col, alpha, r)
        np.testing.assert_allclose(up, cval, rtol=16 * r * ULP)
    run = exact.ExactRun(rp, col, Fraction(1, n))
    for _ in range(8):
        run.step()
        _, up = run.bounds()
        assert all(u == n - 1 for u in up)


def test_dense_solve_agrees_on_random_graphs():
    """Long iterations converge to numpy.linalg.solve of Eq. (la) (n up to 300)."""
    for seed in range(4):
        rp, col = sg.random_graph(300, 0.03, seed)
        alpha = 1.0 / (1 + sg.max_degree(rp))
        cd = exact.katz_dense(rp, col, alpha)
        lo, up = oracle.bounds(rp, col, alpha, 200)
        np.testing.assert_allclose(lo, cd, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(up, cd, rtol=1e-12, atol=1e-15)


def test_exact_bounds_theorem1_and_lemma2():
    """Exact rationals: l_r <= c <= u_r (Theorem 1), l non-decreasing and u
    non-increasing (Lemma 2), on random undirected and directed graphs."""
    for name, (rp, col), und in small_graphs()[:16]:
        if not _nonempty(rp):
            continue
        alpha = Fraction(1, 1 + sg.max_degree(rp))
        c = exact.katz_exact(rp, col, alpha)
        run = exact.ExactRun(rp, col, alpha, undirected=und)
        prev = None
        for _ in range(7):
            run.step()
            lo, up = run.bounds()
            assert all(l <= cv <= u for l, cv, u in zip(lo, c, up)), name
            if prev is not None:
                assert all(a <= b for a, b in zip(prev[0], lo)), name
                assert all(a >= b for a, b in zip(prev[1], up)), name
            prev = (lo, up)


def test_fp64_oracle_tracks_exact_iterates():
    """The FP64 oracle's l_r, u_r equal the exact rationals within a few ulps per
    iteration (the scaled form is Algorithm 1 in exact arithmetic)."""
    for name, (rp, col), und in small_graphs():
        if not _nonempty(rp):
            continue
        alpha = Fraction(1, 1 + sg.max_degree(rp))
        run = exact.ExactRun(rp, col, alpha, undirected=und)
        for r in range(1, 9):
            run.step()
            lo_e, up_e = run.bounds()
            lo, up = oracle.bounds(rp, col, float(alpha), r, undirected=und)
            tol = (4 * r + 8) * ULP
            np.testing.assert_allclose(lo, [float(v) for v in lo_e], rtol=tol, atol=0)
            np.testing.assert_allclose(up, [float(v) for v in up_e], rtol=tol, atol=0)


def test_foster_recurrence_identity():
    """c_r equals f_r - 1 with f_0 = 1, f_{i+1} = alpha A f_i + 1 (Foster's
    heuristic, Section 2.2 and the remark after the complexity analysis)."""
    rp, col = sg.erdos_renyi(600, 2400, 7)
    n = len(rp) - 1
    alpha = 1.0 / (1 + sg.max_degree(rp))
    dense = np.zeros((n, n))
    for v in range(n):
        dense[v, col[rp[v]:rp[v + 1]]] = 1.0
    f = np.ones(n)
    for r in range(1, 25):
        f = alpha * (dense @ f) + 1.0
        c, _ = oracle.walk_state(rp, col, alpha, r)
        np.testing.assert_allclose(c, f - 1.0, rtol=1e-13, atol=1e-15)


def test_dag_bounds_become_exact():
    """On a DAG omega_i = 0 past the longest path, so l = u = c afterwards."""
    rp, col = sg.random_dag(9, 0.45, 11)
    alpha = Fraction(1, 1 + sg.max_degree(rp))
    c = exact.katz_exact(rp, col, alpha)
    lo, up = oracle.bounds(rp, col, float(alpha), 12, undirected=False)
    np.testing.assert_allclose(lo, [float(v) for v in c], rtol=4 * ULP)
    np.testing.assert_array_equal(lo, up)


# --- the top-k test ---------------------------------------------------------------

def test_converged_matches_pairwise_definition():
    """converged() on M = V is True iff the top-k criterion holds pair by pair
    (brute force over random bound arrays with ties)."""
    rng = np.random.default_rng(5)
    checked = 0
    for trial in range(3000):
        n = int(rng.integers(2, 11))
        k = int(rng.integers(1, n + 1))
        lower = rng.integers(0, 6, n).astype(np.float64) / 4.0
        upper = lower + rng.integers(0, 4, n) / 8.0
        eps = [0.0, 1 / 16, 1 / 4][trial % 3]
        ok, M = K.converged(np.arange(n), lower, upper, k, eps)
        assert ok == exact.topk_separated(lower, upper, k, eps), (lower, upper, k, eps)
        order = sorted(range(n), key=lambda v: (-lower[v], v))
        assert list(M[:k]) == order[:k]
        checked += ok
    assert checked > 50


def test_converged_never_drops_topk_and_deactivation_rule():
    rng = np.random.default_rng(9)
    for _ in range(500):
        n = int(rng.integers(3, 15))
        k = int(rng.integers(1, n))
        lower = rng.random(n)
        upper = lower + rng.random(n) * 0.3
        ok, M = K.converged(np.arange(n), lower, upper, k, 0.05)
        order = sorted(range(n), key=lambda v: (-lower[v], v))
        theta = lower[order[k - 1]]
        kept_tail = set(int(v) for v in M[k:])
        for v in order[k:]:
            assert (v in kept_tail) == (not (upper[v] - 0.05 < theta))


def test_exact_ranking_property():
    """Exact Algorithm 1: the certified top-k is correct up to eps against the
    exact Katz scores (Section 3.1: sorting by lower bounds ranks correctly
    except pairs closer than eps)."""
    for name, (rp, col), und in small_graphs():
        if not _nonempty(rp) or not und:
            continue
        n = len(rp) - 1
        alpha = Fraction(1, 1 + sg.max_degree(rp))
        c = exact.katz_exact(rp, col, alpha)
        for k in (1, 2, n // 2, n):
            for eps in (Fraction(0), Fraction(1, 10 ** 6), Fraction(1, 100)):
                if k < 1:
                    continue
                top, r, status, _ = exact.rank_static_exact(rp, col, alpha, k, eps, max_iter=60)
                if status != 0:
                    continue
                rest = [v for v in range(n) if v not in top]
                for a in range(k):
                    for b in range(a + 1, k):
                        assert c[top[a]] > c[top[b]] - eps
                    for v in rest:
                        assert c[top[a]] > c[v] - eps


def test_fp64_oracle_ranking_matches_exact():
    """FP64 and exact Algorithm 1 certify the same top-k at the same r on small
    graphs (gaps between separated scores are far above FP64 rounding)."""
    agree = 0
    for seed in range(30):
        rp, col = sg.random_graph(12, 0.35, 1000 + seed)
        if not _nonempty(rp):
            continue
        alpha = Fraction(1, 1 + sg.max_degree(rp))
        for k, eps in ((3, Fraction(1, 1000)), (5, Fraction(1, 10 ** 6))):
            top_e, r_e, st_e, _ = exact.rank_static_exact(rp, col, alpha, k, eps, max_iter=80)
            res = oracle.rank_static(rp, col, float(alpha), k, float(eps), max_iter=80)
            if st_e == 0:
                assert res.status == oracle.OK
                assert res.iterations == r_e
                # Position by position the same exact score: nodes with equal
                # scores (automorphic twins) may trade places, as FP64 rounding
                # decides their lower-bound order while exact ties go by id.
                c = exact.katz_exact(rp, col, alpha)
                assert [c[int(v)] for v in res.topk] == [c[v] for v in top_e]
                agree += 1
    assert agree > 20


def test_rank_static_cfg_er_small():
    """Erdos-Renyi, n = 16384, M = 8n: the certified top-100 satisfies the pairwise
    criterion on the oracle's own final bounds and is consistent with a 200-step
    reference score vector."""
    rp, col = sg.erdos_renyi(16384, 131072, 1)
    res = oracle.rank_static(rp, col, None, 100, 0.0)
    assert res.status == oracle.OK
    assert res.active_final == 100
    lo, up = res.lower_all, res.upper_all
    top = res.topk
    assert np.all(lo[top[:-1]] > up[top[1:]])
    assert lo[top[-1]] > res.rest_upper_max
    ref, _ = oracle.walk_state(rp, col, res.alpha, 200)
    assert np.all(np.diff(ref[top]) < 0)
    assert ref[top[-1]] > np.max(np.delete(ref, top))


def test_exact_ties_status():
    """Two automorphic nodes share their Katz score, so eps = 0 can never separate
    them; on a graph whose walks die out (a DAG) the loop ends with W_EXACT_TIES."""
    rp, col = sg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 3], undirected=False)  # 1 and 2 tie
    res = oracle.rank_static(rp, col, 0.25, 3, 0.0, undirected=False)
    assert res.status == oracle.W_EXACT_TIES
    assert list(res.topk[:1]) == [0]
    res = oracle.rank_static(rp, col, 0.25, 3, 1e-9, undirected=False)
    assert res.status == oracle.OK


def test_iteration_limit_status():
    """Undirected automorphic twins never separate at eps = 0: W_ITER_LIMIT."""
    rp, col = sg.star_graph(3)
    res = oracle.rank_static(rp, col, None, 2, 0.0, max_iter=25)
    assert res.status == oracle.W_ITER_LIMIT and res.iterations == 25
    assert res.topk[0] == 0 and res.topk[1] == 1


def test_argument_validation():
    rp, col = sg.cycle_graph(5)
    with pytest.raises(ValueError):
        oracle.rank_static(rp, col, 0.5, 2, 0.0)          # alpha * deg_max = 1
    with pytest.raises(ValueError):
        oracle.rank_static(rp, col, None, 0, 0.0)
    with pytest.raises(ValueError):
        oracle.rank_static(rp, col, None, 6, 0.0)
    with pytest.raises(ValueError):
        oracle.rank_static(rp, col, None, 2, -1.0)


# --- dynamic (Algorithm 2) ----------------------------------------------------------

def _random_batch(rng, rp, col, n, n_ins, n_del):
    src = np.repeat(np.arange(n), np.diff(rp))
    und = [(int(a), int(b)) for a, b in zip(src, col) if a < b]
    existing = set(und)
    dels = [und[i] for i in rng.choice(len(und), size=min(n_del, len(und)), replace=False)]
    ins = set()
    while len(ins) < n_ins:
        a, b = sorted(int(v) for v in rng.integers(0, n, 2))
        if a != b and (a, b) not in existing:
            ins.add((a, b))
    return sorted(ins), dels


@pytest.mark.parametrize("seed", range(6))
def test_dynamic_equals_static_recompute(seed):
    """After each batch the delta-form update reproduces the static iterates on
    the new graph at the same r (Section 4: omega' equals what the static
    algorithm computes on the modified graph)."""
    rng = np.random.default_rng(seed)
    rp, col = sg.erdos_renyi(400, 1600, 20 + seed)
    dmax = sg.max_degree(rp)
    alpha = 1.0 / (dmax + 1 + 8)               # headroom for insertions
    dyn = oracle.DynamicOracle(rp, col, alpha, k=20, eps=1e-9, degree_cap=dmax + 8)
    for batch in range(4):
        ins, dels = _random_batch(rng, dyn.row_ptr, dyn.col, 400, 1 + 7 * batch, 1 + 3 * batch)
        res = dyn.update(ins, dels)
        c_ref, x_ref = oracle.walk_state(dyn.row_ptr, dyn.col, alpha, res.iterations)
        np.testing.assert_allclose(res.c, c_ref, rtol=1e-12, atol=1e-16)
        np.testing.assert_allclose(res.x, x_ref, rtol=1e-10, atol=1e-18)
        st = oracle.rank_static(dyn.row_ptr, dyn.col, alpha, 20, 1e-9)
        assert res.status == oracle.OK
        # Same certified ranking (r may differ: the dynamic r never shrinks).
        assert list(res.topk) == list(st.topk)


def test_dynamic_rejects_bad_batches_atomically():
    rp, col = sg.cycle_graph(8)
    dyn = oracle.DynamicOracle(rp, col, 0.2, k=2, eps=1e-6)
    before = (dyn.row_ptr.copy(), dyn.col.copy(), dyn.c.copy())
    bad = [
        ([(0, 1)], []),              # already present
        ([], [(0, 2)]),              # absent
        ([(3, 3)], []),              # self-loop
        ([(0, 9)], []),              # out of range
        ([(0, 2), (2, 0)], []),      # repeated (undirected)
        ([(0, 2)], [(0, 2)]),        # both
        ([(0, 2), (0, 3), (0, 4)], []),   # deg(0) = 5 -> alpha * 5 >= 1
    ]
    for ins, dels in bad:
        with pytest.raises(oracle.UpdateRejected):
            dyn.update(ins, dels)
        np.testing.assert_array_equal(dyn.row_ptr, before[0])
        np.testing.assert_array_equal(dyn.col, before[1])
        np.testing.assert_array_equal(dyn.c, before[2])


def test_dynamic_reactivation_and_more_iterations():
    """A batch that lifts a low-ranked node into the top-k is certified after the
    update exactly as a static run on the new graph certifies it."""
    rp, col = sg.star_graph(6)                     # centre 0
    extra = sg.path_graph(5)
    n = 7 + 5
    src = np.concatenate([np.repeat(np.arange(7), np.diff(rp)),
                          7 + np.repeat(np.arange(5), np.diff(extra[0]))])
    dst = np.concatenate([col, 7 + extra[1]])
    rp2, col2 = sg.from_edges(n, src, dst, undirected=False)
    alpha = 0.08
    dyn = oracle.DynamicOracle(rp2, col2, alpha, k=2, eps=1e-7)
    ins = [(9, 1), (9, 2), (9, 3), (9, 4)]
    res = dyn.update(ins, [])
    st = oracle.rank_static(dyn.row_ptr, dyn.col, alpha, 2, 1e-7)
    assert list(res.topk) == list(st.topk)
    assert 9 in list(res.topk)


# --- bounds of sampled nodes (graphs too large for the whole-graph run) -------

def _host_fetch(rp, col):
    deg = np.diff(rp)

    def fetch(ids):
        ptr = np.concatenate([[0], np.cumsum(deg[ids])])
        parts = [col[rp[v]:rp[v + 1]] for v in ids]
        return ptr, (np.concatenate(parts) if parts else np.empty(0, dtype=np.int32))
    return fetch


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_local_bounds_walks_match_enumeration(r):
    """Sampled-node walk vectors against brute-force walk enumeration on small
    graphs, directed and undirected: x_r(v) = alpha^r omega_r(v)."""
    for name, (rp, col), und in small_graphs()[:10]:
        if not _nonempty(rp):
            continue
        deg = np.diff(rp)
        n = len(rp) - 1
        alpha = 1.0 / (2.0 + deg.max())
        nodes = np.arange(0, n, 2)
        ns, lo, up, c, s = K.local_bounds(_host_fetch(rp, col), deg, alpha, nodes, r, und)
        omega = exact.walks_bruteforce(rp, col, r)
        want_s = np.array([alpha ** r * omega[v] for v in ns])
        assert np.allclose(s, want_s, rtol=8 * r * ULP, atol=0), (name, r)
        want_c = np.array([sum(alpha ** i * exact.walks_bruteforce(rp, col, i)[v] for i in range(1, r + 1)) for v in ns])
        assert np.allclose(c, want_c, rtol=16 * r * ULP, atol=0), (name, r)


def test_local_bounds_equal_whole_graph_run():
    """On R-MAT 10 (undirected) and a random directed graph, the sampled-node
    bounds are bit for bit the whole-graph oracle's, hubs and isolated nodes
    included."""
    cases = [(sg.rmat(10, seed=1), True), (sg.random_graph(60, 0.1, 5, undirected=False), False)]
    for (rp, col), und in cases:
        deg = np.diff(rp)
        alpha = K.default_alpha(int(deg.max()))
        nodes = np.unique(np.r_[0, 5, np.argmax(deg), np.argmin(deg), len(rp) - 2])
        for r in (1, 2, 3):
            lo, up = K.bounds(rp, col, alpha, r, und)
            ns, l2, u2, _, _ = K.local_bounds(_host_fetch(rp, col), deg, alpha, nodes, r, und)
            assert np.array_equal(ns, nodes)
            assert np.array_equal(l2, lo[ns]) and np.array_equal(u2, up[ns])


def test_local_bounds_regular_closed_form():
    """On a cycle (2-regular) every x_i is (2 alpha)^i and c_r a geometric sum."""
    rp, col = sg.cycle_graph(11)
    deg = np.diff(rp)
    alpha = 0.3
    ns, lo, up, c, s = K.local_bounds(_host_fetch(rp, col), deg, alpha, [3, 7], 3)
    q = 2 * alpha
    assert np.allclose(s, q ** 3, rtol=8 * ULP)
    assert np.allclose(c, q + q ** 2 + q ** 3, rtol=16 * ULP)
    assert np.allclose(lo, c + alpha * s, rtol=4 * ULP)
    gamma = 2 / (1 - 2 * alpha)
    assert np.allclose(up, c + alpha * gamma * s, rtol=4 * ULP)


# --- the other stopping criteria (Section 3.1) ----------------------------------

def _crit_graphs():
    out = []
    for seed in range(8):
        out.append(sg.random_graph(7 + seed % 4, 0.4, 300 + seed))
    out.append(sg.star_graph(6))
    out.append(sg.path_graph(7))
    return out


@pytest.mark.parametrize("criterion", ["ranking", "score", "pair"])
def test_criteria_stop_where_the_exact_definition_first_holds(criterion):
    """The FP64 oracle stops at the first r at which the criterion holds on the
    exact bounds (pairwise definitions, brute force), wherever no pair sits
    within rounding of the eps threshold; its output satisfies the definition
    on the exact Katz scores."""
    code = {"ranking": K.RANKING, "score": K.SCORE, "pair": K.PAIR}[criterion]
    eps = 1e-3
    checked = 0
    for rp, col in _crit_graphs():
        if not _nonempty(rp):
            continue
        n = len(rp) - 1
        alpha = Fraction(1, 2 + sg.max_degree(rp))
        pair = (0, n - 1) if criterion == "pair" else None
        r_ex, run = exact.first_stop_exact(rp, col, alpha, Fraction(eps), criterion, pair)
        res = K.rank_static(rp, col, float(alpha), eps=eps, criterion=code, pair=pair)
        if r_ex is None:
            assert res.status != K.OK
            continue
        # Skip graphs where some pair's margin is within rounding of eps.
        lo, up = run.bounds(r_ex)
        margins = [abs(float(lo[a] - (up[b] - Fraction(eps)))) for a in range(n) for b in range(n) if a != b]
        margins += [abs(float(up[v] - lo[v] - Fraction(eps))) for v in range(n)]
        if min(margins) < 1e-12:
            continue
        checked += 1
        assert res.status == K.OK and res.iterations == r_ex
        c = exact.katz_exact(rp, col, alpha)
        if criterion == "score":
            assert all(abs(Fraction(float(res.lower_all[v])) - c[v]) < Fraction(eps) for v in range(n))
            assert len(res.topk) == n
        else:
            order = [int(v) for v in res.topk]
            assert len(order) == (n if criterion == "ranking" else 2)
            for i in range(len(order)):
                for j in range(i + 1, len(order)):
                    assert c[order[i]] > c[order[j]] - Fraction(eps)
    assert checked >= 3


def test_ranking_criterion_is_topk_with_k_equal_n():
    """Section 3.1: for k = n the top-k criterion reduces to the ranking criterion."""
    for seed in range(4):
        rp, col = sg.rmat(8, seed=seed)
        n = len(rp) - 1
        a = K.rank_static(rp, col, None, n, 1e-4)
        b = K.rank_static(rp, col, None, 5, 1e-4, criterion=K.RANKING)
        assert np.array_equal(a.topk, b.topk) and a.iterations == b.iterations and a.status == b.status


def test_separated_fraction_matches_bruteforce():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(2, 40))
        lo = rng.random(n)
        up = lo + rng.random(n) * rng.choice([0.0, 0.01, 0.5], n)
        lo[rng.integers(0, n, 3)] = lo[0]            # some equal values
        up = np.maximum(up, lo)
        want = exact.separated_pairs_bruteforce(lo.tolist(), up.tolist()) / (n * (n - 1) / 2)
        assert K.separated_fraction(lo, up) == pytest.approx(want, abs=1e-15)
    assert K.separated_fraction(np.array([1.0, 2.0, 3.0]), np.array([1.0, 2.0, 3.0])) == 1.0
    assert K.separated_fraction(np.array([1.0, 1.0]), np.array([2.0, 2.0])) == 0.0


def test_pair_criterion_argument_checks():
    rp, col = sg.cycle_graph(5)
    with pytest.raises(ValueError):
        K.rank_static(rp, col, 0.3, criterion=K.PAIR, pair=(1, 1))
    with pytest.raises(ValueError):
        K.rank_static(rp, col, 0.3, criterion=K.PAIR, pair=(0, 9))


# --- the comparison methods (Foster's heuristic, CG on Eq. (la)) ------------------
def _dense_katz(rp, col, alpha):
    n = len(rp) - 1
    A = np.zeros((n, n))
    for v in range(n):
        A[v, col[rp[v]:rp[v + 1]]] = 1.0
    z = np.linalg.solve(np.eye(n) - alpha * A, np.ones(n))
    return alpha * (A @ z)


def test_foster_iterates_are_the_walk_sums():
    """Foster's iteration stopped after r steps gives c_r (f_r - 1 = c_r)."""
    rp, col = sg.erdos_renyi(400, 1600, 3)
    alpha = 1.0 / (1 + sg.max_degree(rp))
    for r in (1, 2, 5, 11):
        res = oracle.foster(rp, col, alpha, tol=0.0, max_iter=r)
        c, _ = oracle.walk_state(rp, col, alpha, r)
        assert res.iterations == r and not res.converged
        np.testing.assert_allclose(res.scores, c, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("name", ["er", "star", "rmat"])
def test_foster_error_within_its_contraction_bound(name):
    """The Foster map f -> alpha A f + 1 contracts the max-norm by alpha d_max,
    so after stopping with change delta the error is at most
    delta * alpha d_max / (1 - alpha d_max) (plus rounding)."""
    rp, col = {"er": lambda: sg.erdos_renyi(500, 2500, 4), "star": lambda: sg.star_graph(40),
               "rmat": lambda: sg.rmat(9, seed=2)}[name]()
    d = sg.max_degree(rp)
    alpha = 0.9 / d
    res = oracle.foster(rp, col, alpha, tol=1e-7)
    exact_c = _dense_katz(rp, col, alpha)
    assert res.converged and res.residual < 1e-7
    bound = res.residual * alpha * d / (1 - alpha * d)
    assert np.max(np.abs(res.scores - exact_c)) <= bound * (1 + 1e-6) + 1e-12


def test_cg_two_distinct_eigenvalues_two_steps():
    """K_6 has two distinct adjacency eigenvalues (5, -1), so CG on
    (I - alpha A) z = 1 stops after two steps, at the closed form
    c = alpha d / (1 - alpha d) = 5 for alpha = 1/6 (Appendix A)."""
    rp, col = sg.complete_graph(6)
    res = oracle.conjugate_gradient(rp, col, 1.0 / 6.0, tol=1e-14)
    assert res.converged and res.iterations <= 2
    np.testing.assert_allclose(res.scores, 5.0, rtol=1e-14)


@pytest.mark.parametrize("name", ["er", "ba", "rmat"])
def test_cg_matches_direct_solve(name):
    rp, col = {"er": lambda: sg.erdos_renyi(600, 3000, 9), "ba": lambda: sg.barabasi_albert(500, 4, 3),
               "rmat": lambda: sg.rmat(9, seed=5)}[name]()
    alpha = 1.0 / (1 + sg.max_degree(rp))
    res = oracle.conjugate_gradient(rp, col, alpha, tol=1e-13)
    assert res.converged
    np.testing.assert_allclose(res.scores, _dense_katz(rp, col, alpha), rtol=1e-11, atol=1e-14)


def test_cg_and_foster_exact_on_star():
    """Star with L leaves: c(centre) = (1 + alpha) alpha L / (1 - alpha^2 L),
    c(leaf) = alpha (1 + alpha L) / (1 - alpha^2 L), in exact arithmetic."""
    L = 12
    rp, col = sg.star_graph(L)
    alpha = Fraction(1, 1 + L)
    c_exact = exact.katz_exact(rp, col, alpha)
    centre = (1 + alpha) * alpha * L / (1 - alpha * alpha * L)
    leaf = alpha * (1 + alpha * L) / (1 - alpha * alpha * L)
    assert c_exact[0] == centre and all(v == leaf for v in c_exact[1:])
    cg = oracle.conjugate_gradient(rp, col, float(alpha), tol=1e-14)
    fo = oracle.foster(rp, col, float(alpha), tol=1e-13)
    for res in (cg, fo):
        np.testing.assert_allclose(res.scores, [float(v) for v in c_exact], rtol=1e-11)


# --- inbound Katz and directed dynamic graphs ---------------------------------------

@pytest.mark.parametrize("name,g,und", [t for t in small_graphs() if not t[2]])
def test_reverse_graph_counts_walks_ending_at_each_node(name, g, und):
    """Walk counts of the reverse graph are the inbound walk counts of the
    graph (Section 2.1), found by enumerating every walk and tallying its end."""
    rp, col = g
    rt, rc = oracle.reverse_graph(rp, col)
    if not _nonempty(rt):
        pytest.skip("no arcs")
    alpha = 1.0 / (1 + sg.max_degree(rt))
    A = K.adjacency(rt, rc)
    x = np.ones(len(rp) - 1)
    for i in range(1, 6):
        x = K.walk_step(A, x, alpha)
        want = np.array(exact.walks_ending_bruteforce(rp, col, i), dtype=np.float64)
        np.testing.assert_allclose(x / alpha ** i, want, rtol=8 * i * ULP)


def test_reverse_graph_structure():
    """Reversing twice gives the graph back; an undirected graph is its own
    reverse; reversed rows are sorted; in-degrees become out-degrees."""
    for name, (rp, col), und in small_graphs():
        rt, rc = oracle.reverse_graph(rp, col)
        rr, rrc = oracle.reverse_graph(rt, rc)
        np.testing.assert_array_equal(rr, rp)
        np.testing.assert_array_equal(rrc, col)
        if und:
            np.testing.assert_array_equal(rt, rp)
            np.testing.assert_array_equal(rc, col)
        for v in range(len(rt) - 1):
            assert np.all(np.diff(rc[rt[v]:rt[v + 1]]) > 0)
        np.testing.assert_array_equal(np.diff(rt), np.bincount(col, minlength=len(rp) - 1))


def _random_directed_batch(rng, rp, col, n, n_ins, n_del):
    src = np.repeat(np.arange(n), np.diff(rp))
    arcs = [(int(a), int(b)) for a, b in zip(src, col)]
    existing = set(arcs)
    dels = [arcs[i] for i in rng.choice(len(arcs), size=min(n_del, len(arcs)), replace=False)]
    ins = set()
    while len(ins) < n_ins:
        a, b = (int(v) for v in rng.integers(0, n, 2))
        if a != b and (a, b) not in existing:
            ins.add((a, b))
    return sorted(ins), dels


@pytest.mark.parametrize("seed", range(4))
def test_dynamic_directed_equals_static_recompute(seed):
    """Algorithm 2 on a directed graph (the search follows reverse arcs):
    after each batch of arc updates the iterates equal a static run on the new
    graph at the same r, and the certified top-k is the static one."""
    rng = np.random.default_rng(seed)
    rp, col = sg.random_graph(300, 0.02, 70 + seed, undirected=False)
    dmax = sg.max_degree(rp)
    alpha = 1.0 / (dmax + 1 + 8)
    dyn = oracle.DynamicOracle(rp, col, alpha, k=15, eps=1e-9, undirected=False, degree_cap=dmax + 8)
    for batch in range(4):
        ins, dels = _random_directed_batch(rng, dyn.row_ptr, dyn.col, 300, 1 + 6 * batch, 1 + 3 * batch)
        res = dyn.update(ins, dels)
        c_ref, x_ref = oracle.walk_state(dyn.row_ptr, dyn.col, alpha, res.iterations)
        np.testing.assert_allclose(res.c, c_ref, rtol=1e-12, atol=1e-16)
        np.testing.assert_allclose(res.x, x_ref, rtol=1e-10, atol=1e-18)
        st = oracle.rank_static(dyn.row_ptr, dyn.col, alpha, 15, 1e-9, undirected=False)
        assert res.status == oracle.OK
        assert list(res.topk) == list(st.topk)
