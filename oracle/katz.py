"""Plain sequential FP64 oracle for the bound-based Katz ranking.

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests, the smoke
check and the benchmark's CPU baseline may use it.

Paper: van der Grinten et al., "Scalable Katz Ranking Computation in Large Static
and Dynamic Graphs", ESA 2018.  Notation follows the paper:

* c(v) = sum_{i>=1} alpha^i omega_i(v), omega_i(v) = number of walks of length i
  starting at v (Eq. (katz), Section 1).
* omega_i(v) = sum_{v->x in E} omega_{i-1}(x), omega_0 = 1 (Eq. (basic_recurrence),
  Section 3.2).
* lower bound l_r = c_r, improved to c_r + alpha^{r+1} omega_r on undirected
  graphs (Section 3.1); upper bound u_r = c_r + alpha^{r+1} omega_r gamma with
  gamma = deg_max / (1 - alpha deg_max), valid for alpha < 1/deg_max (Theorem 1).
* top-k criterion with epsilon-separation l(w) > u(v) - eps (Definition in
  Section 3.1, Eq. (epsilon_sep)) and the active set M (Algorithm 1).

Number representation (the paper is silent on it): the walk counts are carried
in the scaled form x_r = alpha^r omega_r, computed as x_r = alpha * (A x_{r-1}),
i.e. alpha is applied once after each row sum.  This is Algorithm 1 in exact
arithmetic and keeps the values inside FP64 range.  With s = x_r:
    c_r = c_{r-1} + s,   l_r = c_r + alpha * s (undirected) or c_r,
    u_r = c_r + beta * s with beta = fl(alpha * gamma).
Each row sum runs left to right in CSR order (scipy's CSR mat-vec).

Readings of the paper taken here:
* The loop of Algorithm 1 is a do-while: the first convergence test comes after
  iteration 1 (Theorem 1 needs r >= 1).
* converged() scans i in k+1..|M| (not |V|) and removes M[i].
* Ties in the partial sort are broken by ascending node id.
* eps >= 0 is accepted; eps = 0 is plain separation.
* Besides convergence the loop stops at max_iter (W_ITER_LIMIT) or when the walk
  vector is all zero (the bounds are then exact and a pair that is still not
  separated is a true tie: W_EXACT_TIES).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

OK = 0
W_ITER_LIMIT = 1
W_PRECISION_LIMIT = 2
W_EXACT_TIES = 3

# Stopping criteria (Section 3.1).
TOPK, RANKING, SCORE, PAIR = 0, 1, 2, 3


class UpdateRejected(ValueError):
    """An edge-update batch violates the preconditions of Algorithm 2."""


@dataclass
class OracleResult:
    topk: np.ndarray            # node ids, ordered by (lower desc, id asc)
    lower: np.ndarray           # l_r of the top-k, same order
    upper: np.ndarray           # u_r of the top-k
    iterations: int             # r
    status: int
    rest_upper_max: float       # max u_r over V minus the top-k (-inf if empty)
    active_final: int           # |M| at the end
    alpha: float
    gamma: float
    beta: float
    c: np.ndarray = field(repr=False)          # c_r for every node
    x: np.ndarray = field(repr=False)          # x_r = alpha^r omega_r for every node
    lower_all: np.ndarray = field(repr=False)
    upper_all: np.ndarray = field(repr=False)
    active: np.ndarray = field(repr=False)     # the final active set M, top-k first


def adjacency(row_ptr, col, n=None):
    """A[v, x] = 1 for every arc v -> x (rows are out-neighbours)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_ptr) - 1 if n is None else n
    data = np.ones(col.size, dtype=np.float64)
    return sp.csr_matrix((data, col, row_ptr), shape=(n, n))


def max_degree(row_ptr) -> int:
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    return int(deg.max()) if deg.size else 0


def gamma_beta(alpha: float, dmax: int):
    """gamma = deg_max / (1 - alpha deg_max) (Theorem 1) and beta = fl(alpha gamma)."""
    gamma = dmax / (1.0 - alpha * dmax)
    return gamma, alpha * gamma


def check_alpha(alpha: float, dmax: int):
    """Theorem 1 needs alpha < 1/deg_max."""
    if not (alpha > 0.0) or not (alpha * dmax < 1.0):
        raise ValueError(f"alpha={alpha!r} violates 0 < alpha < 1/deg_max (deg_max={dmax})")


def default_alpha(dmax: int) -> float:
    """alpha = 1/(1 + deg_max), the paper's experimental choice (Section 3.1)."""
    return 1.0 / (1.0 + dmax)


def reverse_graph(row_ptr, col):
    """The reverse graph (every arc v -> x becomes x -> v) as a CSR whose rows
    list their sources in ascending order.  Inbound Katz centrality, which
    counts the walks that end at a node, is the outbound centrality of this
    graph (Section 2.1)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    order = np.lexsort((src, col))           # by target, then by source
    rt_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rt_ptr, col + 1, 1)
    return np.cumsum(rt_ptr), src[order].astype(np.int32)


def walk_step(A, x_prev, alpha):
    """One application of Eq. (basic_recurrence) in scaled form: alpha * (A x)."""
    return alpha * (A @ x_prev)


def node_bounds(c, s, alpha, beta, undirected):
    """l_r and u_r from c_r and s = alpha^r omega_r (Section 3.1, Theorem 1)."""
    lower = c + alpha * s if undirected else c.copy()
    upper = c + beta * s
    return lower, upper


def order_by_lower(M, lower):
    """M sorted by decreasing lower bound, ties by increasing id (partialSort)."""
    return M[np.lexsort((M, -lower[M]))]


def converged(M, lower, upper, k, eps):
    """The top-k convergence test of Algorithm 1.

    Sort M by decreasing lower bound; every node past position k whose upper
    bound satisfies u - eps < l(M[k]) leaves M; if more than k nodes remain the
    ranking is not certified; otherwise every adjacent pair of the top-k must be
    eps-separated: u(M[i]) - eps < l(M[i-1]).  Returns (certified, new M), where
    the new M starts with the top-k in ranking order.
    """
    order = order_by_lower(M, lower)
    theta = lower[order[k - 1]]
    tail = order[k:]
    tail = tail[~(upper[tail] - eps < theta)]
    M_new = np.concatenate([order[:k], tail])
    if M_new.size > k:
        return False, M_new
    top = order[:k]
    not_separated = upper[top[1:]] - eps >= lower[top[:-1]]
    return (not bool(not_separated.any())), M_new


def converged_score(lower, upper, eps):
    """Score criterion (Section 3.1): every node's interval is narrower than
    eps, u - l < eps, so every Katz score is known up to eps."""
    return bool(np.all(upper - lower < eps))


def converged_pair(lower, upper, eps, a, b):
    """Pair criterion (Section 3.1): the two given nodes are eps-separated.
    With w the one ahead by (lower desc, id asc) and v the other:
    l(w) > u(v) - eps.  Returns (separated, (w, v))."""
    w, v = (a, b) if (lower[a] > lower[b] or (lower[a] == lower[b] and a < b)) else (b, a)
    return bool(lower[w] > upper[v] - eps), (w, v)


def separated_fraction(lower, upper):
    """Fraction of the n(n-1)/2 unordered node pairs {w, v} that the bounds
    separate (not only eps-separate): l(w) > u(v) or l(v) > u(w) (the
    "Separation" column of Table 1).  Both cannot hold for one pair, since
    l <= u; so the count is the number of ordered pairs with l(w) > u(v),
    found for each v by a search in the sorted lower bounds."""
    n = lower.size
    if n < 2:
        return 1.0
    srt = np.sort(lower)
    above = n - np.searchsorted(srt, upper, side="right")    # #{w : l(w) > u(v)}
    return float(above.sum()) / (n * (n - 1) / 2)


def _result(M, c, s, r, status, alpha, gamma, beta, undirected, k):
    lower, upper = node_bounds(c, s, alpha, beta, undirected)
    top = M[:k]
    rest = np.ones(c.size, dtype=bool)
    rest[top] = False
    rest_max = float(upper[rest].max()) if rest.any() else float("-inf")
    return OracleResult(topk=top.copy(), lower=lower[top], upper=upper[top],
                        iterations=r, status=status, rest_upper_max=rest_max,
                        active_final=int(M.size), alpha=alpha, gamma=gamma, beta=beta,
                        c=c, x=s, lower_all=lower, upper_all=upper, active=M.copy())


def _validate(n, k, eps, max_iter):
    if not (1 <= k <= n):
        raise ValueError(f"k={k} must lie in [1, n={n}]")
    if not (eps >= 0.0):
        raise ValueError(f"eps={eps!r} must be >= 0")
    if max_iter < 1:
        raise ValueError("max_iter must be >= 1")


def rank_static(row_ptr, col, alpha=None, k=10, eps=0.0, undirected=True,
                max_iter=1000, history=None, criterion=TOPK, pair=None):
    """Algorithm 1 (Section 3.2) with the top-k criterion, or another
    stopping criterion of Section 3.1:

    * RANKING: every node eps-separated from every other; this is the top-k
      criterion with k = n (``k`` is ignored).
    * SCORE: u - l < eps for every node; the result lists every node by
      (lower desc, id asc) (``k`` is ignored).
    * PAIR: the two nodes of ``pair`` are eps-separated; the result lists the
      two by (lower desc, id asc) (``k`` is ignored).

    ``alpha=None`` selects 1/(1 + deg_max).  If ``history`` is a list it receives
    x_0, x_1, ..., x_r (used by the dynamic oracle).
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    dmax = max_degree(row_ptr)
    alpha = default_alpha(dmax) if alpha is None else float(alpha)
    check_alpha(alpha, dmax)
    if criterion == PAIR:
        if pair is None or len(pair) != 2 or not all(0 <= int(q) < n for q in pair) or pair[0] == pair[1]:
            raise ValueError("the pair criterion needs two distinct node ids")
        pair = (int(pair[0]), int(pair[1]))
    elif criterion not in (TOPK, RANKING, SCORE):
        raise ValueError(f"unknown criterion {criterion!r}")
    if criterion != TOPK:
        k = n if criterion in (RANKING, SCORE) else 2
    _validate(n, k, eps, max_iter)
    gamma, beta = gamma_beta(alpha, dmax)
    A = adjacency(row_ptr, col, n)

    x = np.ones(n)                 # x_0 = omega_0 = 1
    c = np.zeros(n)                # c_0 = 0
    M = np.arange(n, dtype=np.int64)
    if history is not None:
        history.append(x.copy())
    r = 0
    while True:
        r += 1
        x = walk_step(A, x, alpha)
        c = c + x
        if history is not None:
            history.append(x.copy())
        lower, upper = node_bounds(c, x, alpha, beta, undirected)
        if criterion == SCORE:
            ok = converged_score(lower, upper, eps)
            M = order_by_lower(np.arange(n, dtype=np.int64), lower)
        elif criterion == PAIR:
            ok, wv = converged_pair(lower, upper, eps, *pair)
            M = np.array(wv, dtype=np.int64)
        else:
            ok, M = converged(M, lower, upper, k, eps)
        if ok:
            status = OK
            break
        if not x.any():
            status = W_EXACT_TIES
            break
        if r >= max_iter:
            status = W_ITER_LIMIT
            break
    return _result(M, c, x, r, status, alpha, gamma, beta, undirected, k)


def walk_state(row_ptr, col, alpha=None, r=1):
    """(c_r, x_r) after exactly r iterations of Algorithm 1, no convergence test."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    dmax = max_degree(row_ptr)
    alpha = default_alpha(dmax) if alpha is None else float(alpha)
    check_alpha(alpha, dmax)
    if r < 1:
        raise ValueError("r must be >= 1")
    A = adjacency(row_ptr, col, n)
    x = np.ones(n)
    c = np.zeros(n)
    for _ in range(r):
        x = walk_step(A, x, alpha)
        c = c + x
    return c, x


def bounds(row_ptr, col, alpha=None, r=1, undirected=True):
    """l_r and u_r of every node after exactly r iterations (no convergence test)."""
    dmax = max_degree(row_ptr)
    alpha = default_alpha(dmax) if alpha is None else float(alpha)
    c, x = walk_state(row_ptr, col, alpha, r)
    _, beta = gamma_beta(alpha, dmax)
    return node_bounds(c, x, alpha, beta, undirected)


# ---------------------------------------------------------------------------
# Dynamic graphs: Algorithm 2 (Section 4) in its delta form.
# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# The comparison methods of the paper (Sections 2.2 and 5).
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    scores: np.ndarray      # Katz score of every node
    iterations: int         # matrix-vector products of the iteration
    converged: bool
    residual: float         # the last tested quantity
    alpha: float


def foster(row_ptr, col, alpha=None, tol=1e-9, max_iter=1000):
    """Foster's heuristic (Section 2.2): f_0 = 1, f_{i+1} = alpha A f_i + 1,
    iterated until the largest change of an entry, max |f_{i+1} - f_i|, is
    below ``tol`` (the reading of its error tolerance taken here) or max_iter
    steps; the Katz vector is f - 1."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    dmax = max_degree(row_ptr)
    alpha = default_alpha(dmax) if alpha is None else float(alpha)
    check_alpha(alpha, dmax)
    A = adjacency(row_ptr, col, n)
    f = np.ones(n)
    it, change, conv = 0, float("inf"), False
    while it < max_iter:
        f_new = alpha * (A @ f) + 1.0
        it += 1
        change = float(np.max(np.abs(f_new - f))) if n else 0.0
        f = f_new
        if change < tol:
            conv = True
            break
    return SolveResult(scores=f - 1.0, iterations=it, converged=conv, residual=change, alpha=alpha)


def conjugate_gradient(row_ptr, col, alpha=None, tol=1e-15, max_iter=1000):
    """Conjugate gradients without preconditioning on Eq. (la),
    (I - alpha A) z = 1, from z = 0 (the textbook iteration of Hestenes and
    Stiefel), until the relative residual ||1 - (I - alpha A) z||_2 / ||1||_2
    is below ``tol`` or max_iter steps; the Katz vector is alpha A z
    (Section 1).  The matrix must be symmetric (undirected graph)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    dmax = max_degree(row_ptr)
    alpha = default_alpha(dmax) if alpha is None else float(alpha)
    check_alpha(alpha, dmax)
    A = adjacency(row_ptr, col, n)
    b = np.ones(n)
    z = np.zeros(n)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    bnorm = float(np.sqrt(b @ b))
    it, res, conv = 0, float(np.sqrt(rr)) / bnorm, False
    while it < max_iter:
        q = p - alpha * (A @ p)
        a = rr / float(p @ q)
        z = z + a * p
        r = r - a * q
        rr_new = float(r @ r)
        it += 1
        res = float(np.sqrt(rr_new)) / bnorm
        if res < tol:
            conv = True
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return SolveResult(scores=alpha * (A @ z), iterations=it, converged=conv, residual=res, alpha=alpha)


def _arc_keys(row_ptr, col, n):
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    return src * n + np.asarray(col, dtype=np.int64)


def _csr_from_keys(keys, n):
    keys = np.sort(keys)
    src, dst = keys // n, keys % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    return np.cumsum(row_ptr), dst.astype(np.int32)


class DynamicOracle:
    """Static run (Algorithm 1) followed by batches of edge updates (Algorithm 2).

    Readings of Algorithm 2 taken here:
    * An update pair (a, b) on an undirected graph denotes both arcs a->b, b->a.
    * The batch is validated first (inserted arcs absent, deleted arcs present,
      no self-loops, no repeats, insertions and deletions disjoint) and rejected
      whole with UpdateRejected, leaving the state unchanged.
    * alpha is fixed at construction; gamma follows the current deg_max.  A batch
      that would make alpha * deg_max >= 1, or deg_max exceed ``degree_cap``
      (0 = no cap beyond Theorem 1), is rejected.
    * The level-by-level update uses S_i, the nodes whose walk counts can change
      at level i (see ``update``); omega'_i equals omega_i outside S_i, and the
      level-i change of every node in S_i is added to its running c_r.
    * Reactivation uses the paper's test u(w) >= min_{x in M} l(x) - eps.
    * Afterwards converged() is evaluated and static iterations continue from r
      until it holds (or max_iter / exact ties stop the loop as in rank_static).
    """

    def __init__(self, row_ptr, col, alpha=None, k=10, eps=0.0, undirected=True,
                 max_iter=1000, degree_cap=0):
        self.n = len(row_ptr) - 1
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64).copy()
        self.col = np.asarray(col, dtype=np.int32).copy()
        self.k, self.eps, self.undirected, self.max_iter = k, eps, undirected, max_iter
        self.degree_cap = degree_cap
        dmax = max_degree(self.row_ptr)
        self.alpha = default_alpha(dmax) if alpha is None else float(alpha)
        if degree_cap and dmax > degree_cap:
            raise ValueError("deg_max already exceeds degree_cap")
        hist = []
        res = rank_static(self.row_ptr, self.col, self.alpha, k, eps, undirected,
                          max_iter, history=hist)
        self.X = hist                                  # x_0 .. x_r
        self.c = res.c.copy()
        self.r = res.iterations
        self.M = res.active.copy()      # the active set after the run
        self.result = res

    # -- helpers -----------------------------------------------------------
    def _arcs(self, pairs):
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        if self.undirected:
            return np.concatenate([pairs, pairs[:, ::-1]])
        return pairs

    def _validate_batch(self, ins, dels):
        n = self.n
        for name, p in (("insert", ins), ("delete", dels)):
            if p.size and (p.min() < 0 or p.max() >= n):
                raise UpdateRejected(f"{name}: node id out of range")
            if p.size and np.any(p[:, 0] == p[:, 1]):
                raise UpdateRejected(f"{name}: self-loop")
        keys_E = _arc_keys(self.row_ptr, self.col, n)
        ka = self._arcs(ins)
        kd = self._arcs(dels)
        ki = ka[:, 0] * n + ka[:, 1]
        kdl = kd[:, 0] * n + kd[:, 1]
        if np.unique(ki).size != ki.size or np.unique(kdl).size != kdl.size:
            raise UpdateRejected("repeated edge inside the batch")
        if np.intersect1d(ki, kdl).size:
            raise UpdateRejected("edge both inserted and deleted")
        if np.isin(ki, keys_E).any():
            raise UpdateRejected("inserted edge already present")
        if not np.isin(kdl, keys_E).all():
            raise UpdateRejected("deleted edge absent")
        new_keys = np.concatenate([keys_E[~np.isin(keys_E, kdl)], ki])
        new_rp, new_col = _csr_from_keys(new_keys, n)
        dmax = max_degree(new_rp)
        if not (self.alpha * dmax < 1.0) or (self.degree_cap and dmax > self.degree_cap):
            raise UpdateRejected("update exceeds the degree cap (alpha * deg_max >= 1)")
        return ka, kd, keys_E, kdl, new_rp, new_col

    # -- Algorithm 2 ---------------------------------------------------------
    def update(self, ins_pairs, del_pairs):
        """Applies one batch (Section 4, Algorithm 2) and re-certifies the top-k.

        The walk vectors of the new graph follow from the old ones level by
        level.  Split the arcs into K = E minus D (kept), I (inserted) and D
        (deleted); the new adjacency is A' = A_K + A_I and the old one
        A = A_K + A_D.  With x_i = alpha A x_{i-1} and x'_i = alpha A' x'_{i-1}
        (x'_0 = x_0 = 1):

            x'_i - x_i = alpha (A_K (x'_{i-1} - x_{i-1}) + A_I x'_{i-1} - A_D x_{i-1}).

        The difference is zero outside S_i, the nodes whose walk counts can
        change at level i: the sources of inserted and deleted arcs, and every
        node with a kept arc into S_{i-1}.  Only those nodes are updated, and
        c_r moves by the sum of their level differences.
        """
        ins = np.asarray(ins_pairs if ins_pairs is not None else [], dtype=np.int64).reshape(-1, 2)
        dels = np.asarray(del_pairs if del_pairs is not None else [], dtype=np.int64).reshape(-1, 2)
        arcs_I, arcs_D, keys_E, kdl, new_rp, new_col = self._validate_batch(ins, dels)
        n, alpha = self.n, self.alpha

        rp_k, col_k = _csr_from_keys(keys_E[~np.isin(keys_E, kdl)], n)
        A_K = adjacency(rp_k, col_k, n)
        A_I = sp.csr_matrix((np.ones(len(arcs_I)), (arcs_I[:, 0], arcs_I[:, 1])), shape=(n, n))
        A_D = sp.csr_matrix((np.ones(len(arcs_D)), (arcs_D[:, 0], arcs_D[:, 1])), shape=(n, n))

        seeds = np.zeros(n, dtype=bool)          # sources of updated arcs
        seeds[arcs_I[:, 0]] = True
        seeds[arcs_D[:, 0]] = True
        S = seeds.copy()                          # S_1
        X_new = [self.X[0]]
        for i in range(1, self.r + 1):
            if i > 1:
                S = seeds | ((A_K @ S.astype(np.float64)) > 0)
            diff_prev = X_new[i - 1] - self.X[i - 1]
            delta = alpha * (A_K @ diff_prev + A_I @ X_new[i - 1] - A_D @ self.X[i - 1])
            assert not np.any(delta[~S]), "level difference outside the affected set"
            x_new = self.X[i].copy()
            x_new[S] = self.X[i][S] + delta[S]
            self.c[S] += x_new[S] - self.X[i][S]
            X_new.append(x_new)
        self.X = X_new

        # The graph is now (E minus D) plus I; gamma follows its largest degree.
        self.row_ptr, self.col = new_rp, new_col
        dmax = max_degree(new_rp)
        gamma, beta = gamma_beta(alpha, dmax)
        lower, upper = node_bounds(self.c, self.X[self.r], alpha, beta, self.undirected)

        # Nodes whose upper bound reaches the smallest lower bound in M, less eps,
        # join M again (the test as Section 4 states it).
        thr = lower[self.M].min() - self.eps
        react = np.nonzero(upper >= thr)[0]
        M = np.union1d(self.M, react).astype(np.int64)

        # Static iterations resume from r until the top-k test holds.
        A = adjacency(new_rp, new_col, n)
        status = OK
        while True:
            ok, M = converged(M, lower, upper, self.k, self.eps)
            if ok:
                status = OK
                break
            if not self.X[self.r].any():
                status = W_EXACT_TIES
                break
            if self.r >= self.max_iter:
                status = W_ITER_LIMIT
                break
            self.r += 1
            x = walk_step(A, self.X[self.r - 1], alpha)
            self.c = self.c + x
            self.X.append(x)
            lower, upper = node_bounds(self.c, x, alpha, beta, self.undirected)
        self.M = M
        self.result = _result(M, self.c.copy(), self.X[self.r].copy(), self.r, status,
                              alpha, gamma, beta, self.undirected, self.k)
        return self.result


# ---------------------------------------------------------------------------
# Bounds of a few sampled nodes of a graph too large for the whole-graph run.
# ---------------------------------------------------------------------------

def local_bounds(fetch_rows, deg, alpha, nodes, r, undirected=True, dmax=None):
    """l_r(v) and u_r(v) of the nodes v in ``nodes`` alone (Theorem 1 after r
    iterations of Eq. (basic_recurrence)), each computed from its own r-hop
    neighbourhood: x_1(w) = alpha deg(w) for any w, and x_i(v) = alpha * (sum
    of x_{i-1} over the row of v, left to right in CSR order), the same
    arithmetic in the same order as ``bounds``, so the values are bit for bit
    those of the whole-graph run.

    ``fetch_rows(ids)`` returns (sub_ptr, sub_col) for a sorted array of node
    ids: the concatenated rows of those nodes and their offsets.  ``deg`` is
    the out-degree of every node; ``dmax`` defaults to its maximum (gamma of
    Theorem 1 depends on the whole graph's maximum degree).

    Returns (nodes sorted, lower, upper, c_r, x_r) as arrays.
    """
    deg = np.asarray(deg)
    dmax = int(deg.max()) if dmax is None else int(dmax)
    check_alpha(alpha, dmax)
    if r < 1:
        raise ValueError("r must be >= 1")
    _, beta = gamma_beta(alpha, dmax)
    nodes = np.unique(np.asarray(nodes, dtype=np.int64))
    # need[i]: the nodes whose x_i is required; rows[v]: the row of v.
    need = {r: nodes}
    rows = {}
    for i in range(r, 1, -1):
        missing = np.array([v for v in need[i].tolist() if v not in rows], dtype=np.int64)
        if missing.size:
            sub_ptr, sub_col = fetch_rows(missing)
            sub_ptr = np.asarray(sub_ptr, dtype=np.int64)
            sub_col = np.asarray(sub_col, dtype=np.int64)
            for j, v in enumerate(missing.tolist()):
                rows[v] = sub_col[sub_ptr[j]:sub_ptr[j + 1]]
        nbrs = [rows[v] for v in need[i].tolist()]
        need[i - 1] = np.union1d(nodes, np.concatenate(nbrs) if nbrs else np.empty(0, dtype=np.int64))
    # x[i] = (ids, values) over need[i].
    x = {1: (need[1], alpha * deg[need[1]].astype(np.float64))}
    for i in range(2, r + 1):
        ids_prev, val_prev = x[i - 1]
        vals = np.empty(need[i].size, dtype=np.float64)
        for j, v in enumerate(need[i].tolist()):
            row = rows[v]
            terms = val_prev[np.searchsorted(ids_prev, row)]
            vals[j] = alpha * (np.cumsum(terms)[-1] if terms.size else 0.0)
        x[i] = (need[i], vals)
    c = np.zeros(nodes.size)
    for i in range(1, r + 1):
        ids, vals = x[i]
        c = c + vals[np.searchsorted(ids, nodes)]
    ids, vals = x[r]
    s = vals[np.searchsorted(ids, nodes)]
    lower, upper = node_bounds(c, s, alpha, beta, undirected)
    return nodes, lower, upper, c, s
