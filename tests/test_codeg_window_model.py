"""A CPU model of the key-window schedule the library uses for exact
complement coreness, checked against the oracle's round-by-round order.

The schedule's premise: keys (remaining degrees) only fall, so if a window
holds every live vertex whose key lies in [L, H] with H the largest live key,
then until the window is exhausted each round's largest key and all its
vertices lie inside the window.  The model runs the same decisions as the
GPU path (window cut by a histogram of the top keys, a one-key window when
that key alone exceeds the cap, rounds inside the window, rounds with many
neighbour visits handed to the whole-GPU path) with small caps so that every
branch is taken, and must reproduce the oracle's permutation exactly.  It
shares no code with the library; it restates the schedule to show that the
decomposition itself is exact."""
import numpy as np
import pytest

import oracle
from paper_1907_08607_amd import graphgen as gg


def adjacency(g):
    n = g.n_u + g.n_v
    nb = [[] for _ in range(n)]
    for u in range(g.n_u):
        for k in range(g.u_off[u], g.u_off[u + 1]):
            v = g.n_u + int(g.u_adj[k])
            nb[u].append(v)
            nb[v].append(u)
    return nb


def windowed_codeg(g, cap, bins, dmax, stats):
    nb = adjacency(g)
    n = len(nb)
    deg = np.array([len(a) for a in nb], dtype=np.int64)
    cur = deg.copy()
    alive = np.ones(n, dtype=bool)
    rank = np.full(n, -1, dtype=np.int64)
    nxt = 0

    def remove(front):  # the round's vertices, in id order
        nonlocal nxt
        for x in front:
            rank[x] = nxt
            nxt += 1
            alive[x] = False
        for x in front:
            for y in nb[x]:
                cur[y] -= 1  # a removed vertex's key is never read again

    while nxt < n:
        live = np.nonzero(alive)[0]
        top = int(cur[live].max())
        hist = np.bincount(top - cur[live], minlength=bins)[:bins]
        over = np.nonzero(np.cumsum(hist) > cap)[0]
        take = int(over[0]) if over.size else bins
        take = max(take, 1)
        take = min(take, top + 1)
        lo = top + 1 - take
        win = [int(x) for x in live if cur[x] >= lo]  # id order
        stats["windows"] += 1
        if len(win) > cap:  # one key only: one round removes it all
            assert all(cur[x] == top for x in win)
            stats["one_key"] += 1
            remove(win)
            continue
        while True:
            keys = [cur[x] for x in win if alive[x]]
            if not keys or max(keys) < lo:
                break
            m = max(keys)
            front = [x for x in win if alive[x] and cur[x] == m]
            # the premise: no live vertex outside the window has this key or more
            assert not any(alive[x] and cur[x] >= m and x not in win for x in range(n))
            if deg[front].sum() > dmax:
                stats["handed_back"] += 1
            else:
                stats["in_window"] += 1
            remove(front)
    return rank


GRAPHS = {
    "er_planted": lambda: gg.workload_er_1k_planted(1),
    "powerlaw": lambda: gg.chung_lu(400, 150, 3000, 2.1, 150, 400, 7),
    "giant": lambda: gg.giant_hubs(600, 60, 2, 400, 2, 5),
    "isolated": lambda: gg.from_edges(300, 40, *np.nonzero(np.random.default_rng(9).random((60, 40)) < 0.1)),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_window_schedule_reproduces_the_order(name):
    g = GRAPHS[name]()
    want = np.asarray(oracle.rank(g, "codeg"), dtype=np.int64)
    stats = {"windows": 0, "one_key": 0, "in_window": 0, "handed_back": 0}
    got = windowed_codeg(g, cap=16, bins=16, dmax=40, stats=stats)
    assert np.array_equal(got, want)
    assert stats["windows"] > 1 and stats["in_window"] > 0


def test_every_branch_is_taken():
    stats = {"windows": 0, "one_key": 0, "in_window": 0, "handed_back": 0}
    for name in sorted(GRAPHS):
        windowed_codeg(GRAPHS[name](), cap=16, bins=16, dmax=40, stats=stats)
    assert stats["one_key"] > 0 and stats["handed_back"] > 0 and stats["in_window"] > 0
