"""The parity contract between a GPU ranking and the oracle's.

Positions i and i+1 of the oracle's top-k are robustly separated when
l(o_i) > u(o_{i+1}) (1 + tau); position k is robustly separated from the rest
when l(o_k) > rest_upper_max (1 + tau).  Maximal runs of positions joined by
non-robust separation form tie groups.  The GPU list must equal the oracle's
position by position outside tie groups and may permute a group; if the last
group is not separated from the rest, its slots may hold any node whose oracle
upper bound reaches l(o_k)(1 - tau).  Every returned interval must intersect
the oracle's interval of that node (widened by tau): both contain c.
"""
import numpy as np


def tie_groups(orc, tau):
    O = np.asarray(orc.topk)
    lo, up = orc.lower_all, orc.upper_all
    k = len(O)
    sep = [bool(lo[O[i]] > up[O[i + 1]] * (1 + tau)) for i in range(k - 1)]
    tail_sep = bool(lo[O[k - 1]] > orc.rest_upper_max * (1 + tau)) if np.isfinite(orc.rest_upper_max) else True
    groups, start = [], 0
    for i in range(k - 1):
        if sep[i]:
            groups.append((start, i + 1))
            start = i + 1
    groups.append((start, k))
    return groups, tail_sep


def assert_topk_parity(gpu_ids, gpu_lo, gpu_up, orc, tau=1e-12, widened=False, check_status=True,
                       gpu_status=None):
    O = np.asarray(orc.topk, dtype=np.int64)
    G = np.asarray(gpu_ids, dtype=np.int64)
    assert G.shape == O.shape
    assert len(set(G.tolist())) == len(G), "duplicate ids in the GPU top-k"
    lo_o, up_o = orc.lower_all, orc.upper_all
    groups, tail_sep = tie_groups(orc, tau)
    for gi, (a, b) in enumerate(groups):
        last = gi == len(groups) - 1
        if last and not tail_sep:
            floor = lo_o[O[-1]] * (1 - tau)
            for v in G[a:b]:
                assert up_o[v] >= floor, f"node {v} cannot belong to the top-k tail group"
            assert set(G[:a].tolist()) == set(O[:a].tolist())
        else:
            assert set(G[a:b].tolist()) == set(O[a:b].tolist()), f"positions {a}..{b - 1} differ"
    glo = np.asarray(gpu_lo, dtype=np.float64)
    gup = np.asarray(gpu_up, dtype=np.float64)
    assert np.all(glo <= gup)
    olo = lo_o[G] * (1 - tau) - 1e-300
    oup = up_o[G] * (1 + tau) + 1e-300
    assert np.all(glo <= oup) and np.all(olo <= gup), "GPU and oracle intervals do not intersect"
    if check_status and gpu_status is not None:
        assert gpu_status == orc.status
    return groups
