"""Pins of the C++/OpenMP oracle (``oracle/katz_ref.cpp``).

It must compute what the numpy oracle computes, bit for bit, at any thread
count (same arithmetic in the same order), and it is run directly through the
same closed forms, the sharpness lemma and the exact certified rankings that
pin the numpy oracle, so a mistake of its own (a dropped term, a wrong index,
a reordered sum) fails here even where the numpy oracle is right.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import cpp, exact
import synthgraph as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
ULP = 2.0 ** -52


@pytest.fixture(scope="module", autouse=True)
def built():
    cpp.build(force=not os.path.exists(cpp.LIB_PATH))


def assert_same(a, b):
    assert a.status == b.status and a.iterations == b.iterations
    assert a.active_final == b.active_final
    np.testing.assert_array_equal(np.asarray(a.topk, np.int64), np.asarray(b.topk, np.int64))
    for f in ("lower", "upper", "c", "x", "lower_all", "upper_all"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert a.rest_upper_max == b.rest_upper_max
    assert (a.alpha, a.gamma, a.beta) == (b.alpha, b.gamma, b.beta)


def cases():
    out = [("er16384_s1", sg.erdos_renyi(16384, 131072, 1), None, 100, 0.0, True, 1000),
           ("er16384_s2", sg.erdos_renyi(16384, 131072, 2), None, 100, 0.0, True, 1000),
           ("rmat12", sg.rmat(12, 16, 0.57, 0.19, 0.19, seed=3), None, 50, 1e-6, True, 1000),
           ("ba", sg.barabasi_albert(3000, 5, 4), 0.3 / 100.0, 30, 1e-9, True, 1000),
           ("star_limit", sg.star_graph(3), None, 2, 0.0, True, 25),
           ("dag_ties", sg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 3], undirected=False), 0.25, 3, 0.0, False, 1000),
           ("directed", sg.random_graph(60, 0.1, 8, undirected=False), None, 7, 1e-9, False, 1000),
           ("k_eq_n", sg.random_graph(40, 0.2, 9), None, 40, 1e-3, True, 1000)]
    for seed in range(6):
        out.append((f"small{seed}", sg.random_graph(6 + seed, 0.4, 40 + seed), None, 3, 1e-12, True, 200))
    return out


@pytest.mark.parametrize("name,g,alpha,k,eps,und,max_iter", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_bitwise_equal_to_numpy_oracle(name, g, alpha, k, eps, und, max_iter):
    rp, col = g
    ref = oracle.rank_static(rp, col, alpha, k, eps, undirected=und, max_iter=max_iter)
    for threads in (1, 0):
        got = cpp.rank_static(rp, col, alpha, k, eps, undirected=und, max_iter=max_iter, threads=threads)
        assert_same(got, ref)


def test_bounds_bitwise_equal():
    rp, col = sg.rmat(11, 16, 0.57, 0.19, 0.19, seed=6)
    for r in (1, 2, 7):
        for und in (True, False):
            lo, up = cpp.bounds(rp, col, None, r, undirected=und, threads=3)
            lo_o, up_o = oracle.bounds(rp, col, None, r, undirected=und)
            assert np.array_equal(lo, lo_o) and np.array_equal(up, up_o)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["graph"])
def test_closed_forms_bracketed(case):
    """The closed-form Katz scores of tests/golden lie inside every iterate's
    bounds and the bounds close on them (Theorem 1, Eq. (la))."""
    g = case["graph"]
    if g == "complete":
        (rp, col), und = sg.complete_graph(case["n"]), True
    elif g == "cycle":
        (rp, col), und = sg.cycle_graph(case["n"]), True
    elif g == "star":
        (rp, col), und = sg.star_graph(case["leaves"]), True
    else:
        (rp, col), und = sg.path_graph(case["n"], undirected=False), False
    n = len(rp) - 1
    alpha = float(Fraction(case["alpha"]))
    if case["node"] == "all":
        vals = case["katz"] if isinstance(case["katz"], list) else [case["katz"]] * n
        items = [(v, float(Fraction(x))) for v, x in enumerate(vals)]
    elif case["node"] == "centre":
        items = [(0, float(Fraction(case["katz"])))]
    else:
        items = [(v, float(Fraction(case["katz"]))) for v in range(1, n)]
    for r in (1, 2, 3, 5, 8, 13, 21, 34):
        lo, up = cpp.bounds(rp, col, alpha, r, undirected=und)
        for v, cv in items:
            tol = 8 * r * ULP * max(cv, 1e-300)
            assert lo[v] <= cv + tol and cv - tol <= up[v], (r, v)
    lo, up = cpp.bounds(rp, col, alpha, 400, undirected=und)
    for v, cv in items:
        assert abs(lo[v] - cv) <= 1e-12 * max(1.0, cv)


@pytest.mark.parametrize("n", [4, 6, 9])
def test_sharpness_complete_graph(n):
    """On K_n (and alpha = 1/n) the upper bound equals c = n - 1 at every r."""
    rp, col = sg.complete_graph(n)
    for r in range(1, 20):
        _, up = cpp.bounds(rp, col, 1.0 / n, r)
        np.testing.assert_allclose(up, n - 1.0, rtol=16 * r * ULP)


def test_ranking_matches_exact_algorithm():
    """Same certified top-k, same r, as Algorithm 1 in rational arithmetic."""
    agree = 0
    for seed in range(20):
        rp, col = sg.random_graph(12, 0.35, 2000 + seed)
        if sg.max_degree(rp) == 0:
            continue
        alpha = Fraction(1, 1 + sg.max_degree(rp))
        top_e, r_e, st_e, _ = exact.rank_static_exact(rp, col, alpha, 4, Fraction(1, 10 ** 6), max_iter=80)
        res = cpp.rank_static(rp, col, float(alpha), 4, 1e-6, max_iter=80, threads=2)
        if st_e == 0:
            assert res.status == 0 and res.iterations == r_e
            c = exact.katz_exact(rp, col, alpha)
            assert [c[int(v)] for v in res.topk] == [c[v] for v in top_e]
            agree += 1
    assert agree > 10


def test_certified_topk_is_pairwise_separated():
    """On the plain-method workload (ER, n = 16384, M = 8n, k = 100, eps = 0) the
    output satisfies the pairwise top-k criterion on its own final bounds."""
    rp, col = sg.erdos_renyi(16384, 131072, 3)
    res = cpp.rank_static(rp, col, None, 100, 0.0)
    assert res.status == 0 and res.active_final == 100
    lo, up, top = res.lower_all, res.upper_all, res.topk
    assert np.all(lo[top[:-1]] > up[top[1:]])
    assert lo[top[-1]] > res.rest_upper_max
    assert res.rest_upper_max == np.max(np.delete(up, top))


def test_argument_errors():
    rp, col = sg.cycle_graph(5)
    for kw in (dict(alpha=0.5, k=2), dict(k=0), dict(k=6), dict(k=2, eps=-1.0), dict(k=2, max_iter=0)):
        with pytest.raises(ValueError):
            cpp.rank_static(rp, col, **kw)
    with pytest.raises(ValueError):
        cpp.bounds(rp, col, None, 0)


def test_walk_rows_is_one_iteration_of_the_walk():
    rp, col = sg.rmat(11, 16, 0.57, 0.19, 0.19, seed=7)
    n = len(rp) - 1
    alpha = 1.0 / (1 + sg.max_degree(rp))
    _, x1 = oracle.walk_state(rp, col, alpha, 1)
    _, x2 = oracle.walk_state(rp, col, alpha, 2)
    assert np.array_equal(cpp.walk_rows(rp, col, alpha, 0, n, np.ones(n), threads=1), x1)
    assert np.array_equal(cpp.walk_rows(rp, col, alpha, 100, 900, x1, threads=4), x2[100:900])


def test_thread_count_of_one_call_does_not_stick():
    """A call with threads > 0 uses that many threads for itself only: a later
    call with threads = 0 runs on OpenMP's default again."""
    from oracle import cpp as ocpp
    before = ocpp.max_threads()
    rp, col = sg.erdos_renyi(2000, 8000, 3)
    ocpp.walk_rows(rp, col, 0.01, 0, 100, np.ones(2000), threads=1)
    ocpp.rank_static(rp, col, None, 5, 0.0, threads=1)
    ocpp.bounds(rp, col, None, 2, threads=1)
    assert ocpp.max_threads() == before
