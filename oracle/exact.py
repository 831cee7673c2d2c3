"""Exact-arithmetic counterparts and plain definitions used to pin the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``walks_bruteforce``: omega_i(v) by enumerating every walk (depth-first), the
  definition of omega in Section 1, independent of Eq. (basic_recurrence).
* ``katz_exact``: the closed form of Eq. (la): solve (I - alpha A) z = 1 by
  Gaussian elimination over the rationals, then c = alpha A z.
* ``katz_dense``: the same closed form in FP64 via numpy.linalg.solve.
* ``rank_static_exact``: Algorithm 1 with integer walk counts omega_i and
  rational alpha, c_r, l_r, u_r (no rounding anywhere).
* ``topk_separated``: the top-k criterion of Section 3.1 evaluated pair by pair
  from its definition (every top-k pair eps-separated, and every top-k node
  eps-separated from every other node), without the active set or the
  adjacent-pair shortcut of converged().
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _rows(row_ptr, col):
    row_ptr = [int(v) for v in row_ptr]
    col = [int(v) for v in col]
    return [col[row_ptr[v]:row_ptr[v + 1]] for v in range(len(row_ptr) - 1)]


def walks_bruteforce(row_ptr, col, length):
    """Number of walks with ``length`` arcs starting at each node, by enumeration."""
    rows = _rows(row_ptr, col)

    def count(v, remaining):
        if remaining == 0:
            return 1
        return sum(count(x, remaining - 1) for x in rows[v])

    return [count(v, length) for v in range(len(rows))]


def walks_ending_bruteforce(row_ptr, col, length):
    """Number of walks with ``length`` arcs that end at each node, by
    enumerating every walk from every start (inbound walk counts, Section 2.1)."""
    rows = _rows(row_ptr, col)
    out = [0] * len(rows)

    def walk(v, remaining):
        if remaining == 0:
            out[v] += 1
            return
        for x in rows[v]:
            walk(x, remaining - 1)

    for v in range(len(rows)):
        walk(v, length)
    return out


def katz_exact(row_ptr, col, alpha):
    """c = alpha A (I - alpha A)^{-1} 1 in rational arithmetic (Eq. (la))."""
    alpha = Fraction(alpha)
    rows = _rows(row_ptr, col)
    n = len(rows)
    # Augmented matrix [I - alpha A | 1].
    mat = [[Fraction(int(i == j)) for j in range(n)] + [Fraction(1)] for i in range(n)]
    for v, nbrs in enumerate(rows):
        for x in nbrs:
            mat[v][x] -= alpha
    for p in range(n):
        piv = next(i for i in range(p, n) if mat[i][p] != 0)
        mat[p], mat[piv] = mat[piv], mat[p]
        inv = 1 / mat[p][p]
        mat[p] = [a * inv for a in mat[p]]
        for i in range(n):
            if i != p and mat[i][p] != 0:
                f = mat[i][p]
                mat[i] = [a - f * b for a, b in zip(mat[i], mat[p])]
    z = [mat[i][n] for i in range(n)]
    return [alpha * sum(z[x] for x in nbrs) for nbrs in rows]


def katz_dense(row_ptr, col, alpha):
    """FP64 closed form via numpy.linalg.solve (Eq. (la))."""
    rows = _rows(row_ptr, col)
    n = len(rows)
    A = np.zeros((n, n))
    for v, nbrs in enumerate(rows):
        for x in nbrs:
            A[v, x] += 1.0
    z = np.linalg.solve(np.eye(n) - alpha * A, np.ones(n))
    return alpha * (A @ z)


def topk_separated(lower, upper, k, eps):
    """The top-k criterion from its definition, for the ranking by (lower desc, id asc).

    Returns True iff every pair inside the top-k is eps-separated in ranking
    order and every top-k node is eps-separated from every node outside it.
    """
    n = len(lower)
    order = sorted(range(n), key=lambda v: (-lower[v], v))
    top, rest = order[:k], order[k:]
    for a in range(k):
        for b in range(a + 1, k):
            if not lower[top[a]] > upper[top[b]] - eps:
                return False
        for v in rest:
            if not lower[top[a]] > upper[v] - eps:
                return False
    return True


class ExactRun:
    """Algorithm 1 in exact arithmetic; keeps every iterate for inspection."""

    def __init__(self, row_ptr, col, alpha, undirected=True):
        self.rows = _rows(row_ptr, col)
        self.n = len(self.rows)
        self.alpha = Fraction(alpha)
        self.dmax = max((len(r) for r in self.rows), default=0)
        if not (0 < self.alpha and self.alpha * self.dmax < 1):
            raise ValueError("alpha must satisfy 0 < alpha < 1/deg_max")
        self.gamma = Fraction(self.dmax) / (1 - self.alpha * self.dmax)
        self.undirected = undirected
        self.omega = [[1] * self.n]                  # omega_0 = 1
        self.c = [[Fraction(0)] * self.n]            # c_0 = 0

    def step(self):
        """Iteration r: omega_r by Eq. (basic_recurrence), then c_r."""
        prev = self.omega[-1]
        w = [sum(prev[x] for x in nbrs) for nbrs in self.rows]
        r = len(self.omega)
        a_r = self.alpha ** r
        self.omega.append(w)
        self.c.append([cv + a_r * wv for cv, wv in zip(self.c[-1], w)])

    def bounds(self, r=None):
        """l_r, u_r of every node (Section 3.1, Theorem 1)."""
        r = len(self.omega) - 1 if r is None else r
        a_next = self.alpha ** (r + 1)
        lower = [cv + (a_next * wv if self.undirected else 0)
                 for cv, wv in zip(self.c[r], self.omega[r])]
        upper = [cv + a_next * wv * self.gamma for cv, wv in zip(self.c[r], self.omega[r])]
        return lower, upper


def converged_exact(M, lower, upper, k, eps):
    """converged() of Algorithm 1 on Python lists (exact values)."""
    order = sorted(M, key=lambda v: (-lower[v], v))
    theta = lower[order[k - 1]]
    keep = order[:k] + [v for v in order[k:] if not (upper[v] - eps < theta)]
    if len(keep) > k:
        return False, keep
    for i in range(1, k):
        if upper[keep[i]] - eps >= lower[keep[i - 1]]:
            return False, keep
    return True, keep


def rank_static_exact(row_ptr, col, alpha, k, eps=0, undirected=True, max_iter=200):
    """Algorithm 1 with the top-k criterion, exact.  Returns (top-k, r, status, run)
    where status 0 = certified, 1 = iteration limit, 3 = exact ties."""
    run = ExactRun(row_ptr, col, alpha, undirected)
    eps = Fraction(eps)
    M = list(range(run.n))
    while True:
        run.step()
        r = len(run.omega) - 1
        lower, upper = run.bounds()
        ok, M = converged_exact(M, lower, upper, k, eps)
        if ok:
            return M[:k], r, 0, run
        if not any(run.omega[-1]):
            return M[:k], r, 3, run
        if r >= max_iter:
            return M[:k], r, 1, run


def criterion_holds_exact(lower, upper, eps, criterion, pair=None):
    """The stopping criteria of Section 3.1 from their pairwise definitions,
    on exact values, by brute force over all pairs:
    ranking: every two nodes are eps-separated (the one with the larger lower
    bound, ties by id, ahead); score: u - l < eps for every node; pair: the two
    given nodes are eps-separated."""
    n = len(lower)
    eps = Fraction(eps)

    def sep(a, b):
        w, v = (a, b) if (lower[a] > lower[b] or (lower[a] == lower[b] and a < b)) else (b, a)
        return lower[w] > upper[v] - eps

    if criterion == "ranking":
        return all(sep(a, b) for a in range(n) for b in range(a + 1, n))
    if criterion == "score":
        return all(upper[v] - lower[v] < eps for v in range(n))
    if criterion == "pair":
        return sep(*pair)
    raise ValueError(criterion)


def first_stop_exact(row_ptr, col, alpha, eps, criterion, pair=None, undirected=True, max_iter=200):
    """The first r >= 1 at which the criterion holds on the exact bounds, or None."""
    run = ExactRun(row_ptr, col, alpha, undirected)
    for r in range(1, max_iter + 1):
        run.step()
        lower, upper = run.bounds()
        if criterion_holds_exact(lower, upper, eps, criterion, pair):
            return r, run
        if not any(run.omega[-1]):
            return None, run
    return None, run


def separated_pairs_bruteforce(lower, upper):
    """Unordered pairs {w, v} with l(w) > u(v) or l(v) > u(w), counted one by one."""
    n = len(lower)
    return sum(1 for a in range(n) for b in range(a + 1, n) if lower[a] > upper[b] or lower[b] > upper[a])
