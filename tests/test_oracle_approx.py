"""Pins of the oracle's sparsification (Section 4.6 "Approximate counting"),
CPU only.  The generator is pinned to SplitMix64's published outputs; the kept
graph's count is checked against an independent characterisation (the
original graph's butterflies that survive the draw, enumerated by brute
force); the estimates are checked for unbiasedness over many seeds."""
import math
from itertools import combinations

import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg

M64 = 2**64


def test_splitmix_published_outputs():
    # SplitMix64 started at state 0: its first three outputs as published
    # with the generator (Steele, Lea and Flood, OOPSLA 2014, reference code)
    assert oracle.splitmix(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.splitmix(0, 2) == 0x06C45D188009454F


def butterflies(g):
    """Every butterfly (u1, u2, v1, v2) of g with its four edge positions."""
    off, adj = g.u_off, g.u_adj
    pos = {}
    for u in range(g.n_u):
        for e in range(off[u], off[u + 1]):
            pos[(u, int(adj[e]))] = e
    out = []
    for u1, u2 in combinations(range(g.n_u), 2):
        common = sorted(set(adj[off[u1]:off[u1 + 1]].tolist()) & set(adj[off[u2]:off[u2 + 1]].tolist()))
        for v1, v2 in combinations(common, 2):
            out.append((u1, u2, v1, v2, (pos[(u1, v1)], pos[(u1, v2)], pos[(u2, v1)], pos[(u2, v2)])))
    return out


@pytest.mark.parametrize("kind", ["edge", "color"])
def test_p_one_keeps_everything(kind):
    g = gg.er(60, 50, 700, 3)
    k = oracle.sparsify(g, kind, 1.0, 11)
    assert np.array_equal(k.u_off, g.u_off) and np.array_equal(k.u_adj, g.u_adj)
    c, est, kept = oracle.count_approx(g, kind, 1.0, 11)
    assert c == oracle.count(g, False, False)[0] and est == c and kept == g.m


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("p", [0.5, 0.3])
def test_edge_kept_count_is_surviving_butterflies(seed, p):
    g = gg.random_small(14, 12, 0.45, seed)
    k = oracle.sparsify(g, "edge", p, seed + 100)
    kept_edges = set()
    for u in range(g.n_u):
        for v in k.u_adj[k.u_off[u]:k.u_off[u + 1]]:
            kept_edges.add((u, int(v)))
    pos_kept = {e for u in range(g.n_u) for e in range(g.u_off[u], g.u_off[u + 1])
                if (u, int(g.u_adj[e])) in kept_edges}
    surviving = sum(1 for b in butterflies(g) if all(e in pos_kept for e in b[4]))
    assert oracle.count(k, False, False)[0] == surviving
    # kept rows stay strictly increasing subsets of the input rows
    for u in range(g.n_u):
        row = k.u_adj[k.u_off[u]:k.u_off[u + 1]]
        assert np.all(np.diff(row.astype(np.int64)) > 0)
        assert set(row.tolist()) <= set(g.u_adj[g.u_off[u]:g.u_off[u + 1]].tolist())


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("p", [0.5, 0.34])
def test_color_kept_count_is_monochromatic_butterflies(seed, p):
    g = gg.random_small(14, 12, 0.5, seed)
    k = oracle.sparsify(g, "color", p, seed + 7)
    c = math.ceil(1.0 / p)
    colour = lambda i: (oracle.splitmix(seed + 7, i) * c) >> 64
    mono = sum(1 for (u1, u2, v1, v2, _) in butterflies(g)
               if colour(u1) == colour(u2) == colour(g.n_u + v1) == colour(g.n_u + v2))
    assert oracle.count(k, False, False)[0] == mono
    for u in range(g.n_u):
        for v in k.u_adj[k.u_off[u]:k.u_off[u + 1]]:
            assert colour(u) == colour(g.n_u + int(v))


def test_scale_factors():
    assert oracle.scale("edge", 0.5) == 16.0
    assert oracle.scale("color", 0.5) == 8.0     # 2 colours
    assert oracle.scale("color", 0.3) == 64.0    # ceil(1/0.3) = 4 colours
    assert oracle.scale("edge", 1.0) == oracle.scale("color", 1.0) == 1.0


@pytest.mark.parametrize("kind,p", [("edge", 0.5), ("color", 0.5), ("color", 0.25)])
def test_estimates_are_unbiased(kind, p):
    g = gg.er(200, 150, 3000, 1)
    exact = oracle.count(g, False, False)[0]
    est = np.array([oracle.count_approx(g, kind, p, s)[1] for s in range(300)])
    se = est.std(ddof=1) / math.sqrt(len(est))
    assert abs(est.mean() - exact) < 4.5 * se, (est.mean(), exact, se)


def test_keep_fractions():
    g = gg.er(400, 300, 20000, 5)
    for p in (0.1, 0.5, 0.9):
        kept = oracle.sparsify(g, "edge", p, 3).m
        sd = math.sqrt(g.m * p * (1 - p))
        assert abs(kept - p * g.m) < 5 * sd
    # colours: each vertex's colour is uniform over c, so an edge survives
    # with probability 1/c
    for p in (0.5, 0.25):
        c = math.ceil(1 / p)
        kept = oracle.sparsify(g, "color", p, 9).m
        assert abs(kept - g.m / c) < 0.1 * g.m / c


def test_oracle_rejects_bad_p():
    g = gg.er(10, 10, 20, 1)
    for bad in (0.0, -0.5, float("nan")):
        with pytest.raises(ValueError):
            oracle.sparsify(g, "edge", bad, 1)
