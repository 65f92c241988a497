"""Pins of the oracle's tip decomposition (vertex peeling, Section 3.2 and
Algorithm 5), CPU only.  The tip number of a vertex x of the peeled side X is
the largest k such that some set S of X vertices containing x has, in the
subgraph induced by S and the whole other side, at least k butterflies at
every vertex of S.  On tiny graphs that maximum is found by brute force over
every S and compared with the peeling; closed forms and compositions pin the
rest."""
from itertools import combinations

import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg


def per_vertex_butterflies(adj_sets, S):
    """b(x) for x in S, counting butterflies whose two X vertices are in S."""
    b = {x: 0 for x in S}
    for x, y in combinations(sorted(S), 2):
        c = len(adj_sets[x] & adj_sets[y])
        t = c * (c - 1) // 2
        b[x] += t
        b[y] += t
    return b


def brute_tips(g, side):
    if side == "u":
        adj_sets = [set(g.u_adj[g.u_off[u]:g.u_off[u + 1]].tolist()) for u in range(g.n_u)]
    else:
        adj_sets = [set() for _ in range(g.n_v)]
        for u in range(g.n_u):
            for v in g.u_adj[g.u_off[u]:g.u_off[u + 1]]:
                adj_sets[int(v)].add(u)
    nx = len(adj_sets)
    best = [0] * nx
    for mask in range(1, 1 << nx):
        S = [x for x in range(nx) if mask >> x & 1]
        b = per_vertex_butterflies(adj_sets, S)
        k = min(b.values())
        for x in S:
            best[x] = max(best[x], k)
    return best


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("side", ["u", "v"])
def test_tips_equal_brute_force(seed, side):
    g = gg.random_small(9, 8, 0.5, seed)
    got, _ = oracle.tip(g, side)
    base = 0 if side == "u" else g.n_u
    nx = g.n_u if side == "u" else g.n_v
    assert got[base:base + nx].tolist() == brute_tips(g, side)
    other = got[g.n_u:] if side == "u" else got[:g.n_u]
    assert (other == -1).all()


@pytest.mark.parametrize("a,b", [(2, 2), (3, 4), (5, 3), (6, 6)])
def test_complete_bipartite(a, b):
    # every U vertex is in (a-1)*C(b,2) butterflies, all peeled in one round
    g = gg.complete(a, b)
    got, rounds = oracle.tip(g, "u")
    assert (got[:a] == (a - 1) * b * (b - 1) // 2).all() and rounds == 1


def test_disjoint_union_keeps_each_part():
    g1, g2 = gg.random_small(8, 7, 0.55, 1), gg.complete(4, 5)
    u = gg.disjoint_union(g1, g2)
    t1, _ = oracle.tip(g1, "u")
    t2, _ = oracle.tip(g2, "u")
    tu, _ = oracle.tip(u, "u")
    assert tu[:g1.n_u].tolist() == t1[:g1.n_u].tolist()
    assert tu[g1.n_u:g1.n_u + g2.n_u].tolist() == t2[:g2.n_u].tolist()


def test_tip_at_most_butterfly_count_and_monotone_in_peeling():
    g = gg.er(60, 40, 600, 3)
    t, rounds = oracle.tip(g, "u")
    b = oracle.count(g, want_edge=False)[1]
    assert (t[:g.n_u] <= b[:g.n_u]).all() and (t[:g.n_u] >= 0).all()
    assert rounds >= 1


def test_auto_side_is_fewest_wedges():
    g = gg.er(50, 200, 800, 2)  # V vertices have small degree: U endpoints give fewer wedges
    du = np.diff(g.u_off)
    dv = np.bincount(g.u_adj, minlength=g.n_v)
    su = int((dv * (dv - 1) // 2).sum())
    sv = int((du * (du - 1) // 2).sum())
    t, _ = oracle.tip(g, "auto")
    peeled_u = (t[:g.n_u] >= 0).all()
    assert peeled_u == (su <= sv)
