"""CPU oracle for certified top-k Katz ranking (van der Grinten, Bergamini, Green,
Bader, Meyerhenke, "Scalable Katz Ranking Computation in Large Static and Dynamic
Graphs", ESA 2018).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1807_03847_amd``) never imports it, and this package never imports the
product: the two share no code.  Inputs come from ``synthgraph``, which holds no
Katz arithmetic.

Modules:
  ``katz``    plain, slow, sequential FP64 implementation of the static bound
              iteration (Section 3, Algorithm 1) and of the dynamic update
              (Section 4, Algorithm 2) in its delta form, and the paper's two
              comparison methods (Foster's heuristic, conjugate gradients on
              Eq. (la)).
  ``cpp``     the static part of ``katz`` in C++ with OpenMP (``katz_ref.cpp``),
              bit for bit the same results at any thread count, for graphs the
              numpy form cannot hold (R-MAT scale 27) and for the CPU baseline.
  ``exact``   the same algorithms in exact rational arithmetic for tiny graphs,
              plus the definitions the algorithms are pinned against: the
              closed form of Eq. (la), brute-force walk enumeration, and the
              pairwise definition of the top-k criterion.

Every function is pinned by tests under ``tests/`` (``-m "not gpu"``); none is
"parity unpinned".
"""
from .katz import (OK, W_ITER_LIMIT, W_PRECISION_LIMIT, W_EXACT_TIES,  # noqa: F401
                   OracleResult, rank_static, bounds, walk_state, DynamicOracle,
                   UpdateRejected, foster, conjugate_gradient, SolveResult, reverse_graph)
