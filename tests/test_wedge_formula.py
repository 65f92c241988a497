"""CPU check of the closed form the wedge-count call uses (Algorithm 2's
retrieved wedges): W(rank) = sum over vertices y of h*d - h*(h+1)/2, with d =
deg(y) and h = the neighbours of y ranked above y.  Evaluated here with numpy
and compared with the oracle's wedge counter, which walks the wedges source by
source, for every ordering kind."""
import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg


def closed_form(g, rank):
    u = np.repeat(np.arange(g.n_u), np.diff(g.u_off))
    v = g.n_u + g.u_adj.astype(np.int64)
    n = g.n_u + g.n_v
    above_u = rank[v] < rank[u]  # edge end at u: its neighbour v is ranked above u
    h = np.bincount(u[above_u], minlength=n) + np.bincount(v[~above_u], minlength=n)
    d = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    h, d = h.astype(object), d.astype(object)
    return int(sum(h * d - h * (h + 1) // 2))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kind", sorted(oracle.RANK_KINDS))
def test_closed_form_equals_oracle_wedges(seed, kind):
    g = gg.random_small(30 + seed, 25, 0.2 + 0.05 * seed, seed) if seed < 3 else gg.er(300, 200, 2500, seed)
    r = oracle.rank(g, kind)
    assert closed_form(g, r.astype(np.int64)) == oracle.wedges(g, r)


def test_side_order_closed_form():
    # U-first side order: every V vertex has all its neighbours above it
    g = gg.er(120, 90, 900, 4)
    r = oracle.rank(g, "side_u")
    dv = np.bincount(g.u_adj, minlength=g.n_v).astype(object)
    assert oracle.wedges(g, r) == int(sum(dv * (dv - 1) // 2))
